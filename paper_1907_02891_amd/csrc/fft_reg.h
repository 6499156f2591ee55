// Register-resident mixed-radix transforms with compile-time sizes.
//
// A transform of length N = R0 * R1 * R2 is done in three Stockham passes of
// large radix; each pass runs an R-point DFT entirely in registers, built at
// compile time from 2/3/4/5/8-point kernels by Cooley-Tukey splitting with
// constant internal twiddles.  Data stay in registers; LDS is only the
// exchange buffer between passes (two exchanges per transform), padded by one
// word in 32 against bank conflicts; an exchange may go through it in two
// halves (real parts, then imaginary parts) to halve its size.  Pass twiddles come from FP32 tables
// generated in FP64 on the host.
#pragma once

#include <utility>

#include "fft_lds.h"

namespace lp {

// ------------------------------------------------------------------------
// Compile-time cos/sin of 2 pi m / n: exact integer reduction to an octant,
// then Taylor series in double for the remaining angle in [0, pi/4].
struct CPair {
    double c, s;
};

constexpr double kQuarterPi = 0.785398163397448309615660845819875721;

constexpr double taylor_sin(double x)
{
    double t = x, s = x;
    for (int n = 1; n < 24; ++n) {
        t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        s += t;
    }
    return s;
}

constexpr double taylor_cos(double x)
{
    double t = 1.0, s = 1.0;
    for (int n = 1; n < 24; ++n) {
        t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        s += t;
    }
    return s;
}

constexpr CPair cexp2pi(long m, long n)
{
    m %= n;
    if (m < 0) m += n;
    const long m8 = 8 * m, o = m8 / n;
    const double phi = (o % 2 == 0) ? kQuarterPi * double(m8 - o * n) / double(n)
                                    : kQuarterPi * double((o + 1) * n - m8) / double(n);
    const double cp = taylor_cos(phi), sp = taylor_sin(phi);
    switch (o) {
        case 0: return {cp, sp};
        case 1: return {sp, cp};
        case 2: return {-sp, cp};
        case 3: return {-cp, sp};
        case 4: return {-cp, -sp};
        case 5: return {-sp, -cp};
        case 6: return {sp, -cp};
        default: return {cp, -sp};
    }
}

// a * exp(-/+ 2 pi i M / R) with M, R compile-time; trivial angles skip the
// multiply.
template <int M, int R, bool INV>
__device__ __forceinline__ float2 twc(float2 a)
{
    constexpr int m = ((M % R) + R) % R;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (2 * m == R) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * m == R) {
        return rot<INV>(a);
    } else if constexpr (4 * m == 3 * R) {
        return rot<!INV>(a);
    } else {
        constexpr CPair e = cexp2pi(m, R);
        constexpr float c = static_cast<float>(e.c);
        constexpr float s = INV ? static_cast<float>(e.s) : -static_cast<float>(e.s);
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// Compile-time loop: f(std::integral_constant<int, 0>) ... (N-1).
template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int first_factor(int r)
{
    if (r % 4 == 0 && r != 4 && r != 8) return 4;
    if (r % 2 == 0) return 2;
    if (r % 3 == 0) return 3;
    return 5;
}

constexpr bool is_base_radix(int r) { return r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 8; }

// Largest power of p dividing r.
constexpr int pow_part(int r, int p)
{
    int q = 1;
    while (r % p == 0) { r /= p; q *= p; }
    return q;
}

// A factor A of r with gcd(A, r / A) = 1 and 1 < A < r (the power of 2, else
// the power of 3), or 0 if r is a prime power.
constexpr int coprime_factor(int r)
{
    const int a = pow_part(r, 2);
    if (a > 1 && a < r) return a;
    const int b = pow_part(r, 3);
    if (b > 1 && b < r) return b;
    return 0;
}

// y with x y = 1 mod m (m >= 2, gcd(x, m) = 1).
constexpr int inv_mod(int x, int m)
{
    for (int y = 1; y < m; ++y)
        if ((x * y) % m == 1) return y;
    return 0;
}

// In-place R-point DFT of x[0..R-1] (forward sign -, inverse +, unnormalised).
// R = A * B with gcd(A, B) = 1 (prime-factor algorithm, Good-Thomas): with
// n = (B a + A b) mod R and k the residue with k = k1 mod A, k = k2 mod B,
// the kernel w_R^{nk} splits into w_A^{a k1} w_B^{b k2}, so y is a plain
// A x B two-dimensional DFT with no twiddle factors; all index maps are
// compile-time constants.
// Otherwise (a prime power) Cooley-Tukey: n = B a + b, k = k1 + A k2;
// y[k1 + A k2] = sum_b w_B^{b k2} [ w_R^{b k1} sum_a x[B a + b] w_A^{a k1} ].
template <int R, bool INV>
__device__ __forceinline__ void dftc(float2 *x)
{
    if constexpr (R == 1) {
    } else if constexpr (is_base_radix(R)) {
        dft<R, INV>(x);
    } else if constexpr (coprime_factor(R) != 0) {
        constexpr int A = coprime_factor(R), B = R / A;
        constexpr int EA = B * inv_mod(B % A, A), EB = A * inv_mod(A % B, B);  // CRT idempotents
        float2 t[A][B];
#pragma unroll
        for (int a = 0; a < A; ++a) {
#pragma unroll
            for (int b = 0; b < B; ++b) t[a][b] = x[(B * a + A * b) % R];
            dftc<B, INV>(t[a]);
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            float2 w[A];
#pragma unroll
            for (int a = 0; a < A; ++a) w[a] = t[a][k2];
            dftc<A, INV>(w);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) x[(k1 * EA + k2 * EB) % R] = w[k1];
        }
    } else {
        constexpr int A = first_factor(R), B = R / A;
        float2 t[R];
        sfor<B>([&](auto bi) {
            constexpr int b = decltype(bi)::value;
            float2 u[A];
#pragma unroll
            for (int a = 0; a < A; ++a) u[a] = x[B * a + b];
            dftc<A, INV>(u);
            sfor<A>([&](auto ki) {
                constexpr int k1 = decltype(ki)::value;
                t[b * A + k1] = twc<b * k1, R, INV>(u[k1]);
            });
        });
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            float2 w[B];
#pragma unroll
            for (int b = 0; b < B; ++b) w[b] = t[b * A + k1];
            dftc<B, INV>(w);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = w[k2];
        }
    }
}

// ---------------------------------------------------------------- LDS layout
// Each LDS exchange buffer has one of two layouts, chosen so that both the
// writing and the reading pass address it as (per-butterfly base) + (compile-
// time offset) * j -- one address computation per butterfly, immediate
// offsets for its R elements:
//   L == 0: natural, element n at word n;
//   L == Rw > 0 (written by a first pass of radix Rw, whose butterfly i
//           writes elements i*Rw + j): element n at (n / Rw) * pitch(Rw) +
//           n % Rw with an odd row pitch, so that the stride-Rw writes of
//           consecutive lanes fall in different banks.
// With G interleaved transforms, word w of transform g is at w * G + g.
constexpr int lds_pitch(int rw) { return rw | 1; }
constexpr int lds_words(int n, int rw) { return rw ? (n / rw) * lds_pitch(rw) : n; }

// One pass of radix R over a length-N transform, with P = product of the
// radices of earlier passes; G interleaved transforms per workgroup; thread
// (tt, g), tt in [0, TF), takes butterflies i = tt + s * TF.  LIN / LOUT are
// the layouts of the buffer it reads / writes (LOUT must be R when P == 1
// and 0 otherwise).
template <int N, int R, int P, int TF, int G, int LIN, bool JM = false>
struct RegPass {
    static constexpr int RADIX = R;
    static constexpr int NB = N / R;
    static constexpr int S = (NB + TF - 1) / TF;
    static constexpr int LOUT = (P == 1) ? R : 0;
    static_assert(LIN == 0 || NB % LIN == 0, "input layout stride");

    __device__ __forceinline__ static bool valid(int i) { return NB % TF == 0 || i < NB; }

    // inputs of butterfly i: elements i + j * NB
    __device__ __forceinline__ static void load(float2 (&v)[S][R], const float2 *lds, int tt, int g)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tt + s * TF;
            if (valid(i)) {
                if constexpr (LIN == 0) {
                    const float2 *q = lds + i * G + g;
#pragma unroll
                    for (int j = 0; j < R; ++j) v[s][j] = q[j * NB * G];
                } else {
                    constexpr int PITCH = lds_pitch(LIN);
                    const float2 *q = lds + ((i / LIN) * PITCH + i % LIN) * G + g;
#pragma unroll
                    for (int j = 0; j < R; ++j) v[s][j] = q[j * (NB / LIN) * PITCH * G];
                }
            }
        }
    }

    // one component (C = 0: real, 1: imaginary) of the inputs, through a
    // float buffer with the same word layout (exchanges done in two halves):
    // input j of butterfly i at word in_base(i) + j IN_STRIDE, output j at
    // out_base(i) + j OUT_STRIDE (times G)
    static constexpr int IN_STRIDE = (LIN == 0) ? NB : (NB / LIN) * lds_pitch(LIN);
    static constexpr int OUT_STRIDE = (P == 1) ? 1 : P;
    __device__ __forceinline__ static int in_base(int i)
    {
        if constexpr (LIN == 0) return i;
        else return (i / LIN) * lds_pitch(LIN) + i % LIN;
    }
    __device__ __forceinline__ static int out_base(int i)
    {
        if constexpr (P == 1) return i * lds_pitch(R);
        else return (i - i % P) * R + i % P;
    }

    template <int C>
    __device__ __forceinline__ static void load_part(float2 (&v)[S][R], const float *lds, int tt, int g)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tt + s * TF;
            if (valid(i)) {
                const float *q = lds + in_base(i) * G + g;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if constexpr (C == 0) v[s][j].x = q[j * IN_STRIDE * G];
                    else v[s][j].y = q[j * IN_STRIDE * G];
                }
            }
        }
    }

    template <bool INV>
    __device__ __forceinline__ static void twiddle(float2 (&v)[S][R], const float2 *__restrict__ tw, int tt)
    {
        if constexpr (P > 1) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int i = tt + s * TF;
                if (valid(i)) {
                    // table exp(-2 pi i j k / (P R)), k = i mod P: at (j - 1) P + k
                    // (JM) or at k (R - 1) + j - 1
                    constexpr int SJ = JM ? P : 1;
                    const float2 *t = JM ? tw + (i % P) : tw + (i % P) * (R - 1);
#pragma unroll
                    for (int j = 1; j < R; ++j)
                        v[s][j] = INV ? cmulc(v[s][j], t[(j - 1) * SJ]) : cmul(v[s][j], t[(j - 1) * SJ]);
                }
            }
        }
    }

    // the same through a buffer resource over the table (32-bit offsets)
    static constexpr unsigned TABLE_BYTES = static_cast<unsigned>(P) * (R - 1) * 8u;
    template <bool INV>
    __device__ __forceinline__ static void twiddle(float2 (&v)[S][R], lp_rsrc tw, int tt)
    {
        if constexpr (P > 1) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int i = tt + s * TF;
                if (valid(i)) {
                    constexpr unsigned SJ = JM ? P * 8u : 8u;
                    const unsigned t = JM ? static_cast<unsigned>(i % P) * 8u : static_cast<unsigned>(i % P) * ((R - 1) * 8u);
#pragma unroll
                    for (int j = 1; j < R; ++j) {
                        const float2 w = bload2(tw, t + (j - 1) * SJ);
                        v[s][j] = INV ? cmulc(v[s][j], w) : cmul(v[s][j], w);
                    }
                }
            }
        }
    }

    template <bool INV>
    __device__ __forceinline__ static void butterfly(float2 (&v)[S][R], int tt)
    {
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (valid(tt + s * TF)) dftc<R, INV>(v[s]);
    }

    // outputs of butterfly i: element (i - k) R + k + j P, k = i mod P
    __device__ __forceinline__ static void store(const float2 (&v)[S][R], float2 *lds, int tt, int g)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tt + s * TF;
            if (valid(i)) {
                if constexpr (P == 1) {
                    float2 *q = lds + i * lds_pitch(R) * G + g;
#pragma unroll
                    for (int j = 0; j < R; ++j) q[j * G] = v[s][j];
                } else {
                    const int k = i % P;
                    float2 *q = lds + ((i - k) * R + k) * G + g;
#pragma unroll
                    for (int j = 0; j < R; ++j) q[j * P * G] = v[s][j];
                }
            }
        }
    }

    template <int C>
    __device__ __forceinline__ static void store_part(const float2 (&v)[S][R], float *lds, int tt, int g)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tt + s * TF;
            if (valid(i)) {
                float *q = lds + out_base(i) * G + g;
#pragma unroll
                for (int j = 0; j < R; ++j) q[j * OUT_STRIDE * G] = (C == 0) ? v[s][j].x : v[s][j].y;
            }
        }
    }
};

}  // namespace lp
