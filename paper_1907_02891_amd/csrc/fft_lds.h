// Device-side mixed-radix (2/3/4/5/8) Stockham transforms staged in LDS.
//
// A workgroup holds B interleaved transforms of length n in LDS: element n of
// transform b sits at buf[n * B + b] (B a power of two).  Every radix-r pass
// reads its r inputs at stride n/r (Stockham autosort, decimation in time),
// applies the pass twiddles, runs an r-point DFT in registers, and after a
// barrier writes the r outputs at stride p (the product of the earlier
// radices), so the result ends in natural order with no bit reversal.
// Forward passes use exp(-2 pi i ...) (the sign of Eq. 10); inverse passes
// use the conjugates and are unnormalised.
#pragma once

#include "lp_internal.h"

namespace lp {

// Pointers known to address global memory.  A pointer the compiler cannot
// trace to a kernel argument (one read from a device table of batch items,
// or reassigned on some path) is generic, and its loads and stores become
// flat instructions; those count against both the memory and the LDS wait
// counters, so every LDS wait of a pass would also wait for the HBM traffic
// in flight.  Cast to the global address space, they are global loads and
// stores.
template <class T>
using gptr = T __attribute__((address_space(1))) *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p)
{
    return (gptr<T>)p;
}
// float2 load and store through a global pointer of another element type
// (the vector type's own copy operations take generic references)
typedef float lp_f2v __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ float2 gload2(gptr<const T> p)
{
    const lp_f2v v = *(gptr<const lp_f2v>)p;
    return make_float2(v.x, v.y);
}
template <class T>
__device__ __forceinline__ void gstore2(gptr<T> p, float2 x)
{
    const lp_f2v v = {x.x, x.y};
    *(gptr<lp_f2v>)p = v;
}
// streaming (non-temporal) forms, for data a kernel touches once
template <class T>
__device__ __forceinline__ void gstore2_nt(gptr<T> p, float2 x)
{
    const lp_f2v v = {x.x, x.y};
    __builtin_nontemporal_store(v, (gptr<lp_f2v>)p);
}
template <class T>
__device__ __forceinline__ float2 gload2_nt(gptr<const T> p)
{
    const lp_f2v v = __builtin_nontemporal_load((gptr<const lp_f2v>)p);
    return make_float2(v.x, v.y);
}

// Buffer resources: a base address and a size in bytes held in scalar
// registers, so that each access needs only a 32-bit per-lane byte offset
// (no 64-bit address arithmetic per element, fewer vector registers).
// Accesses past the size read zero and write nothing.
typedef __amdgpu_buffer_rsrc_t lp_rsrc;
typedef unsigned lp_u2v __attribute__((__vector_size__(2 * sizeof(unsigned))));  // the builtins' 64-bit type
__device__ __forceinline__ lp_rsrc buffer_rsrc(const void *base, unsigned bytes)
{
    // third descriptor word for raw (unformatted) 32-bit data on gfx9-family parts
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0), static_cast<int>(bytes),
                                             0x00020000);
}
__device__ __forceinline__ float2 bload2(lp_rsrc r, unsigned off)
{
    const lp_u2v v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    float2 f;
    __builtin_memcpy(&f, &v, sizeof f);
    return f;
}
__device__ __forceinline__ float bload1(lp_rsrc r, unsigned off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bstore2(lp_rsrc r, unsigned off, float2 x)
{
    lp_u2v v;
    __builtin_memcpy(&v, &x, sizeof v);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * w
__device__ __forceinline__ float2 cmul(float2 a, float2 w)
{
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
// a * conj(w)
__device__ __forceinline__ float2 cmulc(float2 a, float2 w)
{
    return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
// a * (-i) for the forward sign, a * (+i) for the inverse one.
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------- r-point DFTs
template <bool INV>
__device__ __forceinline__ void dft2(float2 *v)
{
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2 *v)
{
    // y1,2 = x0 - (x1+x2)/2 -/+ i sin(2pi/3) (x1-x2)   (forward)
    const float s3 = 0.866025403784438646763723170752936183f;
    float2 t = cadd(v[1], v[2]);
    float2 d = cscale(csub(v[1], v[2]), s3);
    float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
    float2 r = rot<INV>(d);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 *v)
{
    float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    float2 c = cadd(v[1], v[3]), d = rot<INV>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2 *v)
{
    const float c1 = 0.309016994374947424102293417182819059f;   // cos(2pi/5)
    const float c2 = -0.809016994374947424102293417182819059f;  // cos(4pi/5)
    const float s1 = 0.951056516295153572116439333379382143f;   // sin(2pi/5)
    const float s2 = 0.587785252292473129168705954639072769f;   // sin(4pi/5)
    float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    float2 x0 = v[0];
    float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    float2 q1 = rot<INV>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    float2 q2 = rot<INV>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2 *v)
{
    const float h = 0.707106781186547524400844362104849039f;  // 1/sqrt(2)
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // o[k] *= w8^k with w8 = exp(-/+ i pi/4)
    float2 o1, o3;
    if (!INV) {
        o1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        o3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    } else {
        o1 = make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y));
        o3 = make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y));
    }
    float2 o2 = rot<INV>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 *v)
{
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 5) dft5<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
}

// i mod p and i / p for 0 <= i < 2^15, from a float reciprocal plus one
// correction step (the float quotient is within 1 of the true one there).
__device__ __forceinline__ int mod_p(int i, int p, float inv_p)
{
    int q = __float2int_rz(static_cast<float>(i) * inv_p);
    int r = i - q * p;
    r += (r < 0) ? p : 0;
    r -= (r >= p) ? p : 0;
    return r;
}

// One radix-R pass over B = 2^logb interleaved transforms held in `buf`.
// Work item w = (butterfly i, transform b), w = i * B + b; thread `tid` of
// `nt` takes items tid, tid + nt, ...  Requires n * B <= kEltsPerThread * nt.
template <int R, bool INV>
__device__ __forceinline__ void stockham_pass(float2 *buf, const FftPass &P, int logb,
                                              const float2 *__restrict__ tw, int tid, int nt)
{
    constexpr int S = (kEltsPerThread + R - 1) / R;
    const int nb = P.nb, p = P.p;
    const int items = nb << logb;
    const int bmask = (1 << logb) - 1;
    float2 v[S][R];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int w = tid + s * nt;
        if (w < items) {
            const int i = w >> logb, b = w & bmask;
#pragma unroll
            for (int j = 0; j < R; ++j) v[s][j] = buf[((i + j * nb) << logb) + b];
            if (p > 1) {
                const int k = mod_p(i, p, P.inv_p);
                const float2 *t = tw + P.tw + k * (R - 1);
#pragma unroll
                for (int j = 1; j < R; ++j) {
                    const float2 w8 = t[j - 1];
                    v[s][j] = INV ? cmulc(v[s][j], w8) : cmul(v[s][j], w8);
                }
            }
            dft<R, INV>(v[s]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int w = tid + s * nt;
        if (w < items) {
            const int i = w >> logb, b = w & bmask;
            const int k = (p > 1) ? mod_p(i, p, P.inv_p) : 0;
            const int base = (i - k) * R + k;
#pragma unroll
            for (int j = 0; j < R; ++j) buf[((base + j * p) << logb) + b] = v[s][j];
        }
    }
    __syncthreads();
}

// The same value in a register the optimiser cannot see through: index
// arithmetic derived from it inside a loop is recomputed per iteration instead
// of being hoisted into registers that stay live across the whole loop.
__device__ __forceinline__ int opaque_v(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// ------------------------------------------------- radix 16 on matrix cores
// A radix-16 pass as a dense product on MFMA with split operands and FP32
// accumulation.  In real form the 16-point DFT maps the 32 reals
// (Re x_j, Im x_j) to the 32 reals (Re y_k, Im y_k); v_mfma_f32_16x16x32
// takes one 16 x 32 tile of that matrix (the Re y rows, or the Im y rows)
// times 16 butterflies.  Lane l of a wave works on butterfly l % 16 and holds
// inputs j = 4 g + t, t < 4, g = l / 16, as the K index 8 g + 2 t + (0 re,
// 1 im); the instruction leaves it outputs k = 4 g + t of the same butterfly.
// SPLIT 1: FP16 hi + lo for both operands (3 products per tile); each
// butterfly's inputs are scaled by a power of two so the largest lies in
// [2^14, 2^15), the matrix by 2^14.  SPLIT 2: BF16 x1 + x2 + x3 (6 products
// per tile, terms of total order <= 4).  Dropped terms are near 2^-22
// relative to the butterfly's largest input.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4v_t __attribute__((ext_vector_type(4)));
typedef unsigned u4v_t __attribute__((ext_vector_type(4)));  // one 16-byte fragment

// cos(2 pi m / 16), correctly rounded, by selects (no indexed local array,
// which would live in scratch memory).
__device__ __forceinline__ float cos16(int m)
{
    m &= 15;
    const int f = (m > 8) ? 16 - m : m;  // cos is even: fold to [0, 8]
    const int q = (f > 4) ? 8 - f : f;   // cos(pi - x) = -cos(x): fold to [0, 4]
    const float v = (q == 0) ? 1.f
                  : (q == 1) ? 0.923879532511286756128183189396788933f   // cos(pi/8)
                  : (q == 2) ? 0.707106781186547524400844362104849039f   // cos(pi/4)
                  : (q == 3) ? 0.382683432365089771728459984030398867f   // cos(3pi/8)
                             : 0.f;
    return (f > 4) ? -v : v;
}

template <int SPLIT>
struct MfmaOps;

template <>
struct MfmaOps<1> {
    half8_t ah[2], al[2];  // [0]: Re y rows, [1]: Im y rows
    static constexpr float kMatScale = 16384.f;  // 2^14
    static constexpr int kVecs = 4;              // 16-byte fragments per lane
    __device__ __forceinline__ void load(const u4v_t *f, int lane)
    {
        ah[0] = __builtin_bit_cast(half8_t, f[lane]);
        ah[1] = __builtin_bit_cast(half8_t, f[64 + lane]);
        al[0] = __builtin_bit_cast(half8_t, f[128 + lane]);
        al[1] = __builtin_bit_cast(half8_t, f[192 + lane]);
    }
    __device__ __forceinline__ void store(u4v_t *f, int lane) const
    {
        f[lane] = __builtin_bit_cast(u4v_t, ah[0]);
        f[64 + lane] = __builtin_bit_cast(u4v_t, ah[1]);
        f[128 + lane] = __builtin_bit_cast(u4v_t, al[0]);
        f[192 + lane] = __builtin_bit_cast(u4v_t, al[1]);
    }
    __device__ __forceinline__ void set_matrix(const float (&m)[2][8])
    {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float x = m[r][q] * kMatScale;
                ah[r][q] = static_cast<_Float16>(x);
                al[r][q] = static_cast<_Float16>(x - static_cast<float>(ah[r][q]));
            }
    }
    __device__ __forceinline__ void product(const float (&x)[8], f4v_t &dre, f4v_t &dim) const
    {
        half8_t h, l;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            h[q] = static_cast<_Float16>(x[q]);
            l[q] = static_cast<_Float16>(x[q] - static_cast<float>(h[q]));
        }
        f4v_t d0 = {}, d1 = {};
        d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], h, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], h, d1, 0, 0, 0);
        d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], l, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], l, d1, 0, 0, 0);
        d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[0], h, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[1], h, d1, 0, 0, 0);
        dre = d0;
        dim = d1;
    }
};

template <>
struct MfmaOps<2> {
    bf8_t a[2][3];
    static constexpr float kMatScale = 1.f;
    static constexpr int kVecs = 6;
    __device__ __forceinline__ void load(const u4v_t *f, int lane)
    {
#pragma unroll
        for (int v = 0; v < 6; ++v) a[v / 3][v % 3] = __builtin_bit_cast(bf8_t, f[64 * v + lane]);
    }
    __device__ __forceinline__ void store(u4v_t *f, int lane) const
    {
#pragma unroll
        for (int v = 0; v < 6; ++v) f[64 * v + lane] = __builtin_bit_cast(u4v_t, a[v / 3][v % 3]);
    }
    __device__ __forceinline__ static void split3(const float (&x)[8], bf8_t (&t)[3])
    {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const __bf16 t1 = static_cast<__bf16>(x[q]);
            const float r1 = x[q] - static_cast<float>(t1);
            const __bf16 t2 = static_cast<__bf16>(r1);
            t[0][q] = t1;
            t[1][q] = t2;
            t[2][q] = static_cast<__bf16>(r1 - static_cast<float>(t2));
        }
    }
    __device__ __forceinline__ void set_matrix(const float (&m)[2][8])
    {
        split3(m[0], a[0]);
        split3(m[1], a[1]);
    }
    __device__ __forceinline__ void product(const float (&x)[8], f4v_t &dre, f4v_t &dim) const
    {
        bf8_t t[3];
        split3(x, t);
        f4v_t d0 = {}, d1 = {};
        // terms a_u x_v with u + v <= 4 (1-based): 11 12 21 13 22 31
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3 - u; ++v) {
                d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][u], t[v], d0, 0, 0, 0);
                d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][u], t[v], d1, 0, 0, 0);
            }
        dre = d0;
        dim = d1;
    }
};

// This lane's slices of the two 16 x 32 tiles of the real DFT matrix: row
// k = lane % 16, K index 8 (lane / 16) + q <-> input j = 4 (lane / 16) + q / 2,
// real part for even q, imaginary for odd q.
template <int SPLIT, bool INV>
__device__ __forceinline__ void mfma16_matrix(MfmaOps<SPLIT> &ops, int lane)
{
    const int k = lane & 15, g = lane >> 4;
    float m[2][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int j = 4 * g + (q >> 1);
        const float fr = cos16(k * j);                 // Re exp(-+2 pi i k j / 16)
        const float s = cos16(k * j + 12);             // sin(2 pi k j / 16)
        const float fi = INV ? s : -s;                 // Im exp(-+2 pi i k j / 16)
        m[0][q] = (q & 1) ? -fi : fr;                  // Re y = fr xr - fi xi
        m[1][q] = (q & 1) ? fr : fi;                   // Im y = fi xr + fr xi
    }
    ops.set_matrix(m);
}

// Fragment table of both directions, written once per plan by one wave:
// [forward | inverse] x kVecs x 64 lanes of 16 bytes.
template <int SPLIT>
__device__ __forceinline__ void mfma16_write_fragments(u4v_t *f, int lane)
{
    MfmaOps<SPLIT> ops;
    mfma16_matrix<SPLIT, false>(ops, lane);
    ops.store(f, lane);
    mfma16_matrix<SPLIT, true>(ops, lane);
    ops.store(f + MfmaOps<SPLIT>::kVecs * 64, lane);
}

// One radix-16 Stockham pass on matrix cores over B = 2^logb interleaved
// transforms: butterfly w = (i, b) = (w >> logb, w & (B-1)), 16 per wave per
// chunk, CH chunks per wave.  With at most kEltsPerThread elements per thread
// the items number at most nt * kEltsPerThread / 16 <= nt * CH / 4.  mf: the
// fragment table (mfma16_write_fragments).
template <int SPLIT, bool INV>
__device__ __forceinline__ void mfma16_pass(float2 *buf, const FftPass &P, int logb,
                                            const float2 *__restrict__ tw, int tid, int nt,
                                            const u4v_t *__restrict__ mf)
{
    constexpr int CH = (kEltsPerThread + 3) / 4;
    const int nb = P.nb, p = P.p;
    const int items = nb << logb;
    const int bmask = (1 << logb) - 1;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int c = lane & 15, g = lane >> 4;
    MfmaOps<SPLIT> ops;
    ops.load(mf + (INV ? MfmaOps<SPLIT>::kVecs * 64 : 0), lane);
    const float unscale0 = 1.f / MfmaOps<SPLIT>::kMatScale;
    float2 out[CH][4];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int chunk = wave + ch * nwaves;
        if (chunk * 16 >= items) break;  // uniform over the wave
        const int w = chunk * 16 + c;
        const bool valid = w < items;
        const int i = w >> logb, b = w & bmask;
        const int k = (p > 1) ? mod_p(i, p, P.inv_p) : 0;
        float x[8];
        float amax = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = 4 * g + t;
            float2 v = make_float2(0.f, 0.f);
            if (valid) {
                v = buf[((i + j * nb) << logb) + b];
                if (p > 1 && j > 0) {
                    const float2 tj = tw[P.tw + k * 15 + j - 1];
                    v = INV ? cmulc(v, tj) : cmul(v, tj);
                }
            }
            x[2 * t] = v.x;
            x[2 * t + 1] = v.y;
            amax = fmaxf(amax, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
        float unscale = unscale0;
        if constexpr (SPLIT == 1) {
            amax = fmaxf(amax, __shfl_xor(amax, 16));
            amax = fmaxf(amax, __shfl_xor(amax, 32));
            int e = 0;
            if (amax > 0.f) {
                (void)frexpf(amax, &e);  // amax = f 2^e, f in [0.5, 1)
                e = 15 - e;              // amax 2^(15-e) in [2^14, 2^15)
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = ldexpf(x[q], e);
            unscale = ldexpf(unscale0, -e);
        }
        f4v_t dre, dim;
        ops.product(x, dre, dim);
#pragma unroll
        for (int t = 0; t < 4; ++t) out[ch][t] = make_float2(dre[t] * unscale, dim[t] * unscale);
    }
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int chunk = wave + ch * nwaves;
        if (chunk * 16 >= items) break;
        const int w = chunk * 16 + c;
        if (w < items) {
            const int i = w >> logb, b = w & bmask;
            const int k = (p > 1) ? mod_p(i, p, P.inv_p) : 0;
            const int base = (i - k) * 16 + k;
#pragma unroll
            for (int t = 0; t < 4; ++t) buf[((base + (4 * g + t) * p) << logb) + b] = out[ch][t];
        }
    }
    __syncthreads();
}

// One radix-16 pass on matrix cores inside a register-resident kernel:
// ITEMS butterflies (a multiple of 16) over the NW waves of the workgroup,
// 16 consecutive items per wave-chunk.  ld(w, j) returns input j of item w
// (twiddled); st(w, k, v) takes output k.  As in mfma16_pass, lane l works on
// item 16 chunk + l % 16 with inputs and outputs 4 (l / 16) .. 4 (l / 16) + 3.
// AHEAD: how many chunks' inputs are in flight before a chunk's product (all
// of a wave's chunks for inputs from HBM, so that their loads overlap; fewer
// keeps fewer registers live).
template <int SPLIT, bool INV, int ITEMS, int NW, int AHEAD, class LD, class ST>
__device__ __forceinline__ void mfma16_items(const u4v_t *__restrict__ mf, LD ld, ST st)
{
    static_assert(SPLIT == 1 || SPLIT == 2, "split form");
    static_assert(ITEMS % 16 == 0 && AHEAD >= 1, "whole chunks");
    constexpr int CHUNKS = ITEMS / 16, CH = (CHUNKS + NW - 1) / NW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    float x[CH][8];
    // a chunk exists for this wave (uniform over the wave)
    auto has = [&](int ch) { return CHUNKS % NW == 0 || wave + ch * NW < CHUNKS; };
    auto fetch = [&](int ch) {
        if (has(ch)) {
            const int w = (wave + ch * NW) * 16 + c;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float2 v = ld(w, 4 * g + t);
                x[ch][2 * t] = v.x;
                x[ch][2 * t + 1] = v.y;
            }
        }
    };
    MfmaOps<SPLIT> ops;
    ops.load(mf + (INV ? MfmaOps<SPLIT>::kVecs * 64 : 0), lane);
    auto compute = [&](int ch) {
        if (!has(ch)) return;
        float unscale = 1.f / MfmaOps<SPLIT>::kMatScale;
        if constexpr (SPLIT == 1) {
            // one power-of-two scale per butterfly: its largest input into
            // [2^14, 2^15)
            float amax = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) amax = fmaxf(amax, fabsf(x[ch][q]));
            amax = fmaxf(amax, __shfl_xor(amax, 16));
            amax = fmaxf(amax, __shfl_xor(amax, 32));
            int e = 0;
            if (amax > 0.f) {
                (void)frexpf(amax, &e);
                e = 15 - e;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) x[ch][q] = ldexpf(x[ch][q], e);
            unscale = ldexpf(unscale, -e);
        }
        f4v_t dre, dim;
        ops.product(x[ch], dre, dim);
        const int w = (wave + ch * NW) * 16 + c;
#pragma unroll
        for (int t = 0; t < 4; ++t) st(w, 4 * g + t, make_float2(dre[t] * unscale, dim[t] * unscale));
    };
    constexpr int A = AHEAD < CH ? AHEAD : CH;
#pragma unroll
    for (int ch = 0; ch < A; ++ch) fetch(ch);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        if (ch + A < CH) fetch(ch + A);
        compute(ch);
    }
}

// Whole transform: all passes of `d` in order.  Entry and exit are barriers.
// SPLIT 0: every pass on the vector ALU in FP32; SPLIT 1 or 2: radix-16
// passes on matrix cores with split operands (the plan's factorisation
// then prefers radix 16; mf is the fragment table), the rest as for SPLIT 0.
// nt is a multiple of 64.
template <bool INV, int SPLIT = 0>
__device__ void lds_fft(float2 *buf, const FftDesc &d, int logb, const float2 *__restrict__ tw,
                        int tid, int nt, const void *mf = nullptr)
{
    for (int ps = 0; ps < d.npass; ++ps) {
        const FftPass P = d.pass[ps];
        // thread-index arithmetic is redone per pass rather than hoisted out
        // of the loop into registers live across all passes
        const int t = opaque_v(tid);
        switch (P.radix) {
            case 16:
                if constexpr (SPLIT != 0)
                    mfma16_pass<SPLIT, INV>(buf, P, logb, tw, t, nt, static_cast<const u4v_t *>(mf));
                break;
            case 8: stockham_pass<8, INV>(buf, P, logb, tw, t, nt); break;
            case 4: stockham_pass<4, INV>(buf, P, logb, tw, t, nt); break;
            case 5: stockham_pass<5, INV>(buf, P, logb, tw, t, nt); break;
            case 3: stockham_pass<3, INV>(buf, P, logb, tw, t, nt); break;
            default: stockham_pass<2, INV>(buf, P, logb, tw, t, nt); break;
        }
    }
}

// Workgroup index remap so that consecutive logical tiles run on the same XCD
// (the hardware deals workgroups round-robin over the 8 XCDs, each with its
// own L2): logical = xcd * q + min(xcd, r) + (b / 8), a bijection on [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

// Tile of workgroup b among the tiles of B rows that hold a kept row
// [keep0, keep1), dealt over the XCDs as xcd_tile deals a whole grid; -1
// past the last such tile.  Dealing the whole grid would leave idle the XCDs
// whose contiguous share of tiles lies outside a narrow kept window.
__device__ __forceinline__ int kept_tile(int b, int ntiles, int B, int keep0, int keep1)
{
    const int k0 = keep0 / B, k1 = min(ntiles, (keep1 + B - 1) / B);
    return b < k1 - k0 ? k0 + xcd_tile(b, k1 - k0) : -1;
}

// Copy of elements 0..total-1, element e = tid + k nt to thread tid: CH of a
// thread's elements are loaded (load(e)) before any is stored (store(e, x)),
// so that its global loads are in flight together rather than one load,
// wait and store per element.
template <int CH, class Load, class Store>
__device__ __forceinline__ void staged_copy(int total, int tid, int nt, Load load, Store store)
{
    for (int e0 = tid; e0 < total; e0 += CH * nt) {
        float2 x[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = e0 + k * nt;
            x[k] = (e < total) ? load(e) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = e0 + k * nt;
            if (e < total) store(e, x[k]);
        }
    }
}

}  // namespace lp
