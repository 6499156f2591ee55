// Four-step column stage for padded columns longer than one LDS tile
// (Sec. 2.5 pads each axis to at least n + k - 1; Eq. 9 and Eq. 10 along y).
//
// A column of Py = P1 * P2 complex values does not fit the 160 KiB of LDS
// one workgroup may hold, so it is transformed as a P1 x P2 matrix with
// element n = P2 n1 + n2 and frequency k = k1 + P1 k2 (Cooley and Tukey's
// split of one DFT into two sets of shorter ones, in the "four-step" order
// of Bailey):
//   X[k1 + P1 k2] = sum_n2 w_P2^(n2 k2) [ w_Py^(n2 k1) sum_n1 x[P2 n1 + n2] w_P1^(n1 k1) ],
//   x[P2 n1 + n2] = sum_k1 w_P1^(-n1 k1) [ w_Py^(-n2 k1) sum_k2 X[k1 + P1 k2] w_P2^(-n2 k2) ],
// with w_N = exp(-2 pi i / N).  The inner sum of the forward and of the
// inverse both run over one k1 and all of k2 / n2, so the spectrum product
// between them fuses into one kernel:
//   k_long_fwd  workgroup (v, group of 2^logb consecutive n2): length-P1
//               DFTs of x[P2 n1 + n2] (rows >= ny are the zero padding and
//               are not read), times w_Py^(n2 k1), to T[v][k1][n2];
//   k_long_mid  workgroup (v, k1): length-P2 DFT of T[v][k1][.], product
//               with the spectrum at frequency k1 + P1 k2 (stored in this
//               order, so the read is contiguous), inverse length-P2 DFT,
//               times w_Py^(-n2 k1), back in place (k_long_mid_reg, with
//               the register-resident passes, when P2 has a column
//               specialisation);
//   k_long_inv  workgroup (v, n2 group): inverse length-P1 DFTs, rows
//               n < ny written back to the intermediate.
// The outer transforms are the LDS Stockham passes of the generic kernels
// (radix 2/3/4/5/8, FP32).  HBM traffic is three passes over a Py-long
// scratch column instead of one over the ny stored rows: this path exists
// for sizes the single-tile kernels cannot take, not for speed.  The two
// columns of an interleaved pair share every line of the intermediate and of
// the spectrum, so all three kernels place them on one XCD (xcd_tile): the
// second of the two reads then hits that XCD's L2 and the halves of a line
// written by the inverse kernel meet there, instead of each line crossing
// HBM twice.
#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace lp {

namespace {

__global__ void __launch_bounds__(1024) k_long_fwd(const float2 *__restrict__ W, LongArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int v = xcd_tile(blockIdx.x, gridDim.x), B = 1 << a.logb, n2b = blockIdx.y << a.logb;
    const int lc = a.lc, cm = (1 << lc) - 1;
    const float2 *col = W + ((static_cast<int64_t>(v >> lc) * a.ny) << lc) + (v & cm);
    // slot (n1, b) = n1 B + b holds x[P2 n1 + n2b + b]
    const int total = a.p1 << a.logb;
    staged_copy<8>(total, tid, nt, [&](int e) {
        const int b = e & (B - 1), n1 = e >> a.logb, n2 = n2b + b;
        const int64_t n = static_cast<int64_t>(a.p2) * n1 + n2;
        return (n2 < a.p2 && n < a.ny) ? col[n << lc] : make_float2(0.f, 0.f);
    }, [&](int e, float2 x) { lds[e] = x; });
    __syncthreads();
    lds_fft<false>(lds, a.f1, a.logb, a.tw1, tid, nt);
    float2 *t = a.T + static_cast<int64_t>(v) * a.py;
    for (int e = tid; e < total; e += nt) {
        const int b = e & (B - 1), k1 = e >> a.logb, n2 = n2b + b;
        // n2 k1 <= (P2 - 1)(P1 - 1) < Py: the exponent needs no reduction
        if (n2 < a.p2) t[static_cast<int64_t>(k1) * a.p2 + n2] = cmul(lds[e], a.twq[n2 * k1]);
    }
}

template <int FORM, bool CONJ>
__global__ void __launch_bounds__(1024) k_long_mid(LongArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int v = xcd_tile(blockIdx.x, gridDim.x), k1 = blockIdx.y;
    float2 *t = a.T + static_cast<int64_t>(v) * a.py + static_cast<int64_t>(k1) * a.p2;
    staged_copy<8>(a.p2, tid, nt, [&](int n2) { return t[n2]; }, [&](int n2, float2 x) { lds[n2] = x; });
    __syncthreads();
    lds_fft<false>(lds, a.f2, 0, a.tw2, tid, nt);
    // Eq. 9: X[k1 + P1 k2] times the spectrum, stored row k1 P2 + k2
    const int lc = a.lc, cm = (1 << lc) - 1;
    const int64_t base = ((static_cast<int64_t>(v >> lc) * a.py + static_cast<int64_t>(k1) * a.p2) << lc) + (v & cm);
    staged_copy<8>(a.p2, tid, nt, [&](int k2) {
        const int64_t idx = base + (static_cast<int64_t>(k2) << lc);
        const float2 x = lds[k2];
        if constexpr (FORM == 1) {
            return cscale(x, static_cast<const float *>(a.kh)[idx]);
        } else {
            const float2 k = static_cast<const float2 *>(a.kh)[idx];
            return CONJ ? cmulc(x, k) : cmul(x, k);
        }
    }, [&](int k2, float2 x) { lds[k2] = x; });
    __syncthreads();
    lds_fft<true>(lds, a.f2, 0, a.tw2, tid, nt);
    for (int n2 = tid; n2 < a.p2; n2 += nt) t[n2] = cmulc(lds[n2], a.twq[n2 * k1]);
}

__global__ void __launch_bounds__(1024) k_long_inv(float2 *__restrict__ W, LongArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int v = xcd_tile(blockIdx.x, gridDim.x), B = 1 << a.logb, n2b = blockIdx.y << a.logb;
    const float2 *t = a.T + static_cast<int64_t>(v) * a.py;
    const int total = a.p1 << a.logb;
    staged_copy<8>(total, tid, nt, [&](int e) {
        const int b = e & (B - 1), k1 = e >> a.logb, n2 = n2b + b;
        return (n2 < a.p2) ? t[static_cast<int64_t>(k1) * a.p2 + n2] : make_float2(0.f, 0.f);
    }, [&](int e, float2 x) { lds[e] = x; });
    __syncthreads();
    lds_fft<true>(lds, a.f1, a.logb, a.tw1, tid, nt);
    const int lc = a.lc, cm = (1 << lc) - 1;
    float2 *col = W + ((static_cast<int64_t>(v >> lc) * a.ny) << lc) + (v & cm);
    for (int e = tid; e < total; e += nt) {
        const int b = e & (B - 1), n1 = e >> a.logb, n2 = n2b + b;
        const int64_t n = static_cast<int64_t>(a.p2) * n1 + n2;
        if (n2 < a.p2 && n < a.ny) col[n << lc] = lds[e];
    }
}

}  // namespace

hipError_t launch_long_cols(float2 *W, const LongArgs &a, int ncols, int form, bool conj_k,
                            int threads_outer, int threads_mid, hipStream_t s, int mid_spec,
                            const ColRegArgs *mid)
{
    if (a.p1 < 2 || a.p2 < 2 || static_cast<int64_t>(a.p1) * a.p2 != a.py || a.p2 > kMaxColLen ||
        (a.p1 << a.logb) > kMaxColLen || a.p1 > 65535 || !a.T || !a.kh)
        return hipErrorInvalidValue;
    // the LDS passes need n * B <= kEltsPerThread * threads, threads a multiple of 64
    if ((a.p1 << a.logb) > kEltsPerThread * threads_outer || a.p2 > kEltsPerThread * threads_mid ||
        threads_outer % 64 || threads_mid % 64 || threads_outer > 1024 || threads_mid > 1024)
        return hipErrorInvalidValue;
    const dim3 go(ncols, (a.p2 + (1 << a.logb) - 1) >> a.logb), gm(ncols, a.p1);
    const size_t lo = static_cast<size_t>(a.p1) << a.logb << 3, lm = static_cast<size_t>(a.p2) << 3;
    hipLaunchKernelGGL(k_long_fwd, go, dim3(threads_outer), lo, s, W, a);
    if (mid_spec >= 0) {
        if (!mid) return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if ((e = launch_long_mid_reg(a, *mid, mid_spec, ncols, form, conj_k, s)) != hipSuccess) return e;
    } else if (form == 1) {
        hipLaunchKernelGGL((k_long_mid<1, false>), gm, dim3(threads_mid), lm, s, a);
    } else if (conj_k) {
        hipLaunchKernelGGL((k_long_mid<2, true>), gm, dim3(threads_mid), lm, s, a);
    } else {
        hipLaunchKernelGGL((k_long_mid<2, false>), gm, dim3(threads_mid), lm, s, a);
    }
    hipLaunchKernelGGL(k_long_inv, go, dim3(threads_outer), lo, s, W, a);
    return hipGetLastError();
}

hipError_t set_long_attributes()
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_long_fwd),
        reinterpret_cast<const void *>(&k_long_mid<1, false>),
        reinterpret_cast<const void *>(&k_long_mid<2, false>),
        reinterpret_cast<const void *>(&k_long_mid<2, true>),
        reinterpret_cast<const void *>(&k_long_inv),
    };
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return set_long_mid_attributes();
}

}  // namespace lp
