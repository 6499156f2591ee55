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

// Whole transform: all passes of `d` in order.  Entry and exit are barriers.
template <bool INV>
__device__ void lds_fft(float2 *buf, const FftDesc &d, int logb, const float2 *__restrict__ tw,
                        int tid, int nt)
{
    for (int ps = 0; ps < d.npass; ++ps) {
        const FftPass P = d.pass[ps];
        switch (P.radix) {
            case 8: stockham_pass<8, INV>(buf, P, logb, tw, tid, nt); break;
            case 4: stockham_pass<4, INV>(buf, P, logb, tw, tid, nt); break;
            case 5: stockham_pass<5, INV>(buf, P, logb, tw, tid, nt); break;
            case 3: stockham_pass<3, INV>(buf, P, logb, tw, tid, nt); break;
            default: stockham_pass<2, INV>(buf, P, logb, tw, tid, nt); break;
        }
    }
}

// The same value in a register the optimiser cannot see through: index
// arithmetic derived from it inside a loop is recomputed per iteration instead
// of being hoisted into registers that stay live across the whole loop.
__device__ __forceinline__ int opaque_v(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Workgroup index remap so that consecutive logical tiles run on the same XCD
// (the hardware deals workgroups round-robin over the 8 XCDs, each with its
// own L2): logical = xcd * q + min(xcd, r) + (b / 8), a bijection on [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

}  // namespace lp
