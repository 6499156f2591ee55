// HIP kernels (gfx950) of the FFT convolution hot path and of the kernel
// spectrum.
//
// Hot path (Fig. 1 of Bara et al. 2019: FFT -> pixel-wise product -> iFFT,
// with the zero padding of Sec. 2.5 and the input-sized output of Sec. 3):
//   k_rows_r2c   forward real-to-complex transform of each map row, length Px,
//                with columns >= nx read as zero; writes the Px/2+1 spectrum
//                columns into the blocked intermediate W;
//   k_cols_conv  per block of columns: forward transform of length Py (rows
//                >= ny read as zero), multiply by the stored kernel spectrum
//                (Eq. 9), inverse transform, keep rows < ny (in place in W);
//   k_rows_c2r   inverse complex-to-real transform of each row, keep columns
//                < nx (the crop).
// Intermediate layout: column v of row i sits at
//   W[((v >> logc) * ny + i) << logc | (v & (C-1))],
// C = 2^logc interleaved columns (C = 2 for every plan with two or more
// stored columns): a row stage with B rows per workgroup touches C*B*8-byte
// runs, the column stage reads and writes one column at stride C (the
// workgroup of the neighbouring column takes the other half of each line).
// Real transforms use the half-length trick: z[n] = x[2n] + i x[2n+1] is
// transformed at length M = Px/2 and split with exp(-2 pi i k/Px).
#include <algorithm>

#include "fft_lds.h"

namespace lp {

// ------------------------------------------------------------------- rows fwd
template <int SPLIT>
__global__ void __launch_bounds__(1024) k_rows_r2c(const float *__restrict__ R,
                                                   float2 *__restrict__ W, RowArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int B = 1 << a.logb, C = 1 << a.logc;
    const int row0 = xcd_tile(blockIdx.x, gridDim.x) << a.logb;
    const int m = a.m;

    // Load B rows as z[n] = x[2n] + i x[2n+1]; columns >= nx and rows >= ny
    // are the zero padding and are never read.
    for (int b = 0; b < B; ++b) {
        const int row = row0 + b;
        const float *src = R + static_cast<int64_t>(row) * a.nx;
        staged_copy<8>(m, tid, nt, [&](int n) {
            float x0 = 0.f, x1 = 0.f;
            if (row < a.ny) {
                const int c0 = 2 * n;
                if (c0 < a.nx) x0 = src[c0];
                if (c0 + 1 < a.nx) x1 = src[c0 + 1];
            }
            return make_float2(x0, x1);
        }, [&](int n, float2 x) { lds[(n << a.logb) + b] = x; });
    }
    __syncthreads();
    lds_fft<false, SPLIT>(lds, a.fx, a.logb, a.tw, tid, nt, a.mf);

    // X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[M-k]) / 2,
    // O = -i (Z[k] - conj Z[M-k]) / 2, w = exp(-2 pi i / Px), 0 <= k <= M.
    const int total = a.nblk << (a.logb + a.logc);
    for (int e = tid; e < total; e += nt) {
        const int c = e & (C - 1);
        const int b = (e >> a.logc) & (B - 1);
        const int kb = e >> (a.logc + a.logb);
        const int k = (kb << a.logc) + c;
        const int row = row0 + b;
        if (row >= a.ny) continue;
        float2 X = make_float2(0.f, 0.f);
        if (k < a.h) {
            const int k1 = (k == m) ? 0 : k;
            const int k2 = (k == 0) ? 0 : m - k;
            const float2 z1 = lds[(k1 << a.logb) + b];
            const float2 z2 = lds[(k2 << a.logb) + b];
            const float2 E = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
            const float2 O = make_float2(0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
            X = cadd(E, cmul(O, a.rtw[k]));
        }
        W[((static_cast<int64_t>(kb) * a.ny + row) << a.logc) + c] = X;
    }
}

// ---------------------------------------------------------------- columns
// One column per workgroup.  FORM 1: real even spectrum, one quadrant stored
// (py/2+1 rows per column).  FORM 2: complex spectrum, py rows per column.  CONJ: use conj(Khat) (the
// transposed operator).  ACC > 0: several source classes (Eq. 4); class t's
// block sits a.w_stride elements after class 0's and its spectrum
// a.kh_stride bytes after class 0's; the products are summed in registers
// (at most ACC per thread) before the one inverse transform.
template <int FORM, bool CONJ, int SPLIT, int ACC>
__global__ void __launch_bounds__(1024) k_cols_conv(float2 *__restrict__ W, ColArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    const int py = a.py, ny = a.ny;
    // element i of column v at ((v / C) * ny + i) * C + v % C (C = 2^logc);
    // the spectrum likewise with ku rows
    const int lc = a.logc, cm = (1 << lc) - 1;
    float2 *col = W + ((static_cast<int64_t>(v >> lc) * ny) << lc) + (v & cm);

    // product of element e of this column with one class's spectrum
    auto spec = [&](const void *kh, int e, float2 x) {
        if constexpr (FORM == 1) {
            const float *kq = static_cast<const float *>(kh) + ((static_cast<int64_t>(v >> lc) * a.ku) << lc) + (v & cm);
            const int uq = (2 * e <= py) ? e : py - e;
            return cscale(x, kq[uq << lc]);
        } else {
            const float2 k = (static_cast<const float2 *>(kh) + ((static_cast<int64_t>(v >> lc) * py) << lc) +
                              (v & cm))[e << lc];
            return CONJ ? cmulc(x, k) : cmul(x, k);
        }
    };

    if constexpr (ACC > 0) {
        float2 acc[ACC];
#pragma unroll
        for (int q = 0; q < ACC; ++q) acc[q] = make_float2(0.f, 0.f);
        for (int t = 0; t < a.classes; ++t) {
            const float2 *src = col + t * a.w_stride;
            const void *kh = static_cast<const char *>(a.kh) + t * a.kh_stride;
            __syncthreads();  // the previous class's products are all read
            staged_copy<8>(py, tid, nt, [&](int e) { return (e < ny) ? src[e << lc] : make_float2(0.f, 0.f); },
                           [&](int e, float2 x) { lds[e] = x; });
            __syncthreads();
            lds_fft<false, SPLIT>(lds, a.fy, 0, a.tw, opaque_v(tid), nt, a.mf);
            const int t0 = opaque_v(tid);
#pragma unroll
            for (int q = 0; q < ACC; ++q) {
                const int e = t0 + q * nt;
                if (e < py) acc[q] = cadd(acc[q], spec(kh, e, lds[e]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ACC; ++q) {
            const int e = tid + q * nt;
            if (e < py) lds[e] = acc[q];
        }
    } else {
        staged_copy<8>(py, tid, nt, [&](int e) { return (e < ny) ? col[e << lc] : make_float2(0.f, 0.f); },
                       [&](int e, float2 x) { lds[e] = x; });
        __syncthreads();
        lds_fft<false, SPLIT>(lds, a.fy, 0, a.tw, tid, nt, a.mf);
        staged_copy<8>(py, tid, nt, [&](int e) { return spec(a.kh, e, lds[e]); },
                       [&](int e, float2 x) { lds[e] = x; });
    }
    __syncthreads();
    lds_fft<true, SPLIT>(lds, a.fy, 0, a.tw, tid, nt, a.mf);

    for (int e = tid; e < ny; e += nt) col[e << lc] = lds[e];
}

// ------------------------------------------------------------------- rows inv
template <int SPLIT>
__global__ void __launch_bounds__(1024) k_rows_c2r(const float2 *__restrict__ W,
                                                   float *__restrict__ S, RowArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int B = 1 << a.logb, C = 1 << a.logc;
    const int row0 = xcd_tile(blockIdx.x, gridDim.x) << a.logb;
    const int m = a.m;

    // Stage X[k], 0 <= k <= M, of B rows (slot (k, b) = k * B + b).
    const int total = a.nblk << (a.logb + a.logc);
    staged_copy<8>(total, tid, nt, [&](int e) {
        const int c = e & (C - 1);
        const int b = (e >> a.logc) & (B - 1);
        const int kb = e >> (a.logc + a.logb);
        const int k = (kb << a.logc) + c;
        const int row = row0 + b;
        return (k < a.h && row < a.ny) ? W[((static_cast<int64_t>(kb) * a.ny + row) << a.logc) + c]
                                       : make_float2(0.f, 0.f);
    }, [&](int e, float2 x) {
        const int c = e & (C - 1);
        const int b = (e >> a.logc) & (B - 1);
        const int k = ((e >> (a.logc + a.logb)) << a.logc) + c;
        if (k < a.h) lds[(k << a.logb) + b] = x;
    });
    __syncthreads();

    // Z[k] = (X[k] + conj X[M-k]) + i w^-k (X[k] - conj X[M-k]), 0 <= k < M
    // (twice the spectrum of x[2n] + i x[2n+1]); pairs (k, M-k) are done by
    // one thread, in place, using w^-(M-k) = -w^k.
    const int half = m >> 1;
    const int npair = half + 1;
    for (int e = tid; e < (npair << a.logb); e += nt) {
        const int b = e & (B - 1);
        const int k = e >> a.logb;
        const int k2 = m - k;
        const float2 x1 = lds[(k << a.logb) + b];
        const float2 x2 = lds[(k2 << a.logb) + b];
        const float2 w = a.rtw[k];
        // term for index k: s = x1 + conj x2, d = x1 - conj x2, Z = s + i conj(w) d
        float2 s = make_float2(x1.x + x2.x, x1.y - x2.y);
        float2 d = make_float2(x1.x - x2.x, x1.y + x2.y);
        float2 wd = cmulc(d, w);
        const float2 zk = make_float2(s.x - wd.y, s.y + wd.x);
        if (k2 != k && k2 < m) {
            // term for index M-k: s' = x2 + conj x1, d' = x2 - conj x1,
            // Z = s' + i (-w) d'
            float2 s2 = make_float2(x2.x + x1.x, x2.y - x1.y);
            float2 d2 = make_float2(x2.x - x1.x, x2.y + x1.y);
            float2 wd2 = cmul(d2, w);
            lds[(k2 << a.logb) + b] = make_float2(s2.x + wd2.y, s2.y - wd2.x);
        }
        if (k < m) lds[(k << a.logb) + b] = zk;
    }
    __syncthreads();
    lds_fft<true, SPLIT>(lds, a.fx, a.logb, a.tw, tid, nt, a.mf);

    for (int b = 0; b < B; ++b) {
        const int row = row0 + b;
        if (row >= a.ny) break;
        float *dst = S + static_cast<int64_t>(row) * a.nx;
        for (int n = tid; n < m; n += nt) {
            const int c0 = 2 * n;
            if (c0 >= a.nx) break;
            const float2 z = lds[(n << a.logb) + b];
            dst[c0] = z.x;
            if (c0 + 1 < a.nx) dst[c0 + 1] = z.y;
        }
    }
}

// ----------------------------------------------------------- kernel spectrum
// Direct FP64 DFT of the wrap-centred kernel, separable over the two axes
// (Eq. 10 restricted to the kernel's support): first along x for each kernel
// row, t1(a, v) = sum_b K(a,b) exp(-2 pi i v (b-cx) / Px), 0 <= v < H; then
// along y.  Twiddles come from an exact FP64 table tab[m] = exp(-2 pi i m/N)
// indexed by the product reduced modulo N (kept by incremental addition).
__global__ void __launch_bounds__(256) k_spec_rows(const double *__restrict__ K, int ky, int kx,
                                                   int cx, int px, int h,
                                                   const double2 *__restrict__ tabx,
                                                   double2 *__restrict__ t1)
{
    const int a = blockIdx.y;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= h || a >= ky) return;
    int64_t m0 = (-static_cast<int64_t>(v) * cx) % px;
    int mi = static_cast<int>(m0 < 0 ? m0 + px : m0);
    double re = 0.0, im = 0.0;
    const double *krow = K + static_cast<int64_t>(a) * kx;
    for (int b = 0; b < kx; ++b) {
        const double2 w = tabx[mi];
        const double kv = krow[b];
        re = fma(kv, w.x, re);
        im = fma(kv, w.y, im);
        mi += v;
        if (mi >= px) mi -= px;
    }
    t1[static_cast<int64_t>(a) * h + v] = make_double2(re, im);
}

// Second axis: Khat(u, v) = sum_a t1(a, v) exp(-2 pi i u (a-cy) / Py), scaled,
// rounded once to FP32, written in the blocked layout of the column stage.
// FORM 1 keeps only the real part for 0 <= u <= Py/2 (the spectrum of a
// mirror-symmetric kernel is real and even).  Columns v >= H of the last
// block are written as zero.
__global__ void __launch_bounds__(256) k_spec_cols(const double2 *__restrict__ t1, int ky, int cy,
                                                   int py, int ku, int h, int logc, int nblk,
                                                   const double2 *__restrict__ taby, double scale,
                                                   int form, void *__restrict__ kh, int r0, int p2)
{
    // stored row r; frequency u = r, or k1 + (py / p2) k2 for r = k1 p2 + k2
    // in the four-step order
    const int r = r0 + static_cast<int>(blockIdx.y);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ku || v >= (nblk << logc)) return;
    const int u = p2 ? r / p2 + (py / p2) * (r % p2) : r;
    double re = 0.0, im = 0.0;
    if (v < h) {
        int64_t m0 = (-static_cast<int64_t>(u) * cy) % py;
        int mi = static_cast<int>(m0 < 0 ? m0 + py : m0);
        for (int a = 0; a < ky; ++a) {
            const double2 w = taby[mi];
            const double2 t = t1[static_cast<int64_t>(a) * h + v];
            if (form == 1) {
                re = fma(t.x, w.x, re);
            } else {
                re = fma(t.x, w.x, fma(-t.y, w.y, re));
                im = fma(t.x, w.y, fma(t.y, w.x, im));
            }
            mi += u;
            if (mi >= py) mi -= py;
        }
    }
    const int vb = v >> logc, c = v & ((1 << logc) - 1);
    const int64_t idx = ((static_cast<int64_t>(vb) * ku + r) << logc) + c;
    if (form == 1)
        static_cast<float *>(kh)[idx] = static_cast<float>(re * scale);
    else
        static_cast<float2 *>(kh)[idx] =
            make_float2(static_cast<float>(re * scale), static_cast<float>(im * scale));
}

// ------------------------------------------------- matrix-core fragments
template <int SPLIT>
__global__ void __launch_bounds__(64) k_mfma_fragments(u4v_t *f)
{
    mfma16_write_fragments<SPLIT>(f, threadIdx.x);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_mfma_fragments(int split, void *table, hipStream_t s)
{
    u4v_t *f = static_cast<u4v_t *>(table);
    if (split == 1) hipLaunchKernelGGL(k_mfma_fragments<1>, dim3(1), dim3(64), 0, s, f);
    else if (split == 2) hipLaunchKernelGGL(k_mfma_fragments<2>, dim3(1), dim3(64), 0, s, f);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

static size_t row_lds_bytes(const RowArgs &a) { return static_cast<size_t>(a.m + 1) << a.logb << 3; }

hipError_t launch_rows_r2c(const float *R, float2 *W, const RowArgs &a, int threads, hipStream_t s)
{
    const dim3 g((a.ny + (1 << a.logb) - 1) >> a.logb), t(threads);
    const size_t lds = row_lds_bytes(a);
    switch (a.fx.split) {
        case 1: hipLaunchKernelGGL(k_rows_r2c<1>, g, t, lds, s, R, W, a); break;
        case 2: hipLaunchKernelGGL(k_rows_r2c<2>, g, t, lds, s, R, W, a); break;
        default: hipLaunchKernelGGL(k_rows_r2c<0>, g, t, lds, s, R, W, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_rows_c2r(const float2 *W, float *S, const RowArgs &a, int threads, hipStream_t s)
{
    const dim3 g((a.ny + (1 << a.logb) - 1) >> a.logb), t(threads);
    const size_t lds = row_lds_bytes(a);
    switch (a.fx.split) {
        case 1: hipLaunchKernelGGL(k_rows_c2r<1>, g, t, lds, s, W, S, a); break;
        case 2: hipLaunchKernelGGL(k_rows_c2r<2>, g, t, lds, s, W, S, a); break;
        default: hipLaunchKernelGGL(k_rows_c2r<0>, g, t, lds, s, W, S, a); break;
    }
    return hipGetLastError();
}

template <int SPLIT, int ACC>
static void launch_cols_sum(float2 *W, const ColArgs &a, int form, dim3 g, dim3 t, size_t lds, hipStream_t s)
{
    if (form == 1)
        hipLaunchKernelGGL((k_cols_conv<1, false, SPLIT, ACC>), g, t, lds, s, W, a);
    else
        hipLaunchKernelGGL((k_cols_conv<2, false, SPLIT, ACC>), g, t, lds, s, W, a);
}

template <int SPLIT>
static void launch_cols_split(float2 *W, const ColArgs &a, int form, bool conj_k, bool sum, dim3 g,
                              dim3 t, size_t lds, hipStream_t s)
{
    // class sums: 8 accumulators per thread when they suffice, else kEltsPerThread
    if (sum && a.py <= 8 * static_cast<int>(t.x))
        launch_cols_sum<SPLIT, 8>(W, a, form, g, t, lds, s);
    else if (sum)
        launch_cols_sum<SPLIT, kEltsPerThread>(W, a, form, g, t, lds, s);
    else if (form == 1)
        hipLaunchKernelGGL((k_cols_conv<1, false, SPLIT, 0>), g, t, lds, s, W, a);
    else if (conj_k)
        hipLaunchKernelGGL((k_cols_conv<2, true, SPLIT, 0>), g, t, lds, s, W, a);
    else
        hipLaunchKernelGGL((k_cols_conv<2, false, SPLIT, 0>), g, t, lds, s, W, a);
}

hipError_t launch_cols_conv(float2 *W, const ColArgs &a, int form, bool conj_k, int threads,
                            hipStream_t s, bool class_sum)
{
    if (class_sum && conj_k) return hipErrorInvalidValue;  // class sums are forward only
    if (threads * kEltsPerThread < a.py) return hipErrorInvalidValue;
    const size_t lds = static_cast<size_t>(a.py) << 3;
    const dim3 g(a.ncols), t(threads);
    switch (a.fy.split) {
        case 1: launch_cols_split<1>(W, a, form, conj_k, class_sum, g, t, lds, s); break;
        case 2: launch_cols_split<2>(W, a, form, conj_k, class_sum, g, t, lds, s); break;
        default: launch_cols_split<0>(W, a, form, conj_k, class_sum, g, t, lds, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_spec_rows(const double *K, int ky, int kx, int cx, int px, int h,
                            const double2 *tabx, double2 *t1, hipStream_t s)
{
    const dim3 g((h + 255) / 256, ky), t(256);
    hipLaunchKernelGGL(k_spec_rows, g, t, 0, s, K, ky, kx, cx, px, h, tabx, t1);
    return hipGetLastError();
}

hipError_t launch_spec_cols(const double2 *t1, int ky, int cy, int py, int ku, int h, int logc,
                            int nblk, const double2 *taby, double scale, int form, void *kh,
                            hipStream_t s, int p2)
{
    const int ncol = nblk << logc;
    // grid.y is limited to 65535: stored rows in chunks
    for (int r0 = 0; r0 < ku; r0 += 65535) {
        const dim3 g((ncol + 255) / 256, std::min(65535, ku - r0)), t(256);
        hipLaunchKernelGGL(k_spec_cols, g, t, 0, s, t1, ky, cy, py, ku, h, logc, nblk, taby, scale,
                           form, kh, r0, p2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int SPLIT>
static hipError_t generic_attributes()
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_rows_r2c<SPLIT>),
        reinterpret_cast<const void *>(&k_rows_c2r<SPLIT>),
        reinterpret_cast<const void *>(&k_cols_conv<1, false, SPLIT, 0>),
        reinterpret_cast<const void *>(&k_cols_conv<2, false, SPLIT, 0>),
        reinterpret_cast<const void *>(&k_cols_conv<2, true, SPLIT, 0>),
        reinterpret_cast<const void *>(&k_cols_conv<1, false, SPLIT, 8>),
        reinterpret_cast<const void *>(&k_cols_conv<2, false, SPLIT, 8>),
        reinterpret_cast<const void *>(&k_cols_conv<1, false, SPLIT, kEltsPerThread>),
        reinterpret_cast<const void *>(&k_cols_conv<2, false, SPLIT, kEltsPerThread>),
    };
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_kernel_attributes()
{
    hipError_t e = generic_attributes<0>();
    if (e == hipSuccess) e = generic_attributes<1>();
    if (e == hipSuccess) e = generic_attributes<2>();
    return e;
}

}  // namespace lp

// ===================================================== register-resident columns
#include "fft_reg.h"

namespace lp {

// Chunks of a matrix-core first pass whose inputs are read from HBM before
// the first product: all of a wave's (8 per wave in the 18432-point column
// kernels, 6 in the 9216-point rows; with 3 the continental split column
// stage took 2.10 instead of 1.48 ms).
constexpr int MF_AHEAD_HBM = 8;

// One column per workgroup: forward transform (radices R0, R1, R2), spectrum
// multiply in registers, inverse transform (radices R2, R1, R0; its first
// pass consumes the forward's last-pass outputs straight from registers), and
// only rows < ny read or written.  Intermediate in the column interleave
// C = 2^lc: element i of column v at ((v / C) ny + i) C + v mod C; the result
// goes to the same place in a.wout when it is given (out of place).
// SUM (several source classes, Eq. 4): the forward transform and the product
// with the class's spectrum are repeated for each class t (intermediate
// W + t w_stride, spectrum kh + t kh_stride bytes) and summed in registers
// before the one inverse transform, whose result goes to class 0's column.
// MF (1 or 2): the radix-16 pass R0 (the forward's first, the inverse's
// last) runs on the matrix cores in that split form, reading the column from
// HBM and writing it back.
template <int N, int TF, int R0, int R1, int R2, int OCC, int FORM, bool CONJ, bool SUM, int MF = 0>
__global__ void __launch_bounds__(((TF + 63) / 64) * 64, SUM ? 0 : OCC) k_cols_reg(float2 *__restrict__ W, ColRegArgs a,
                                                                         const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    constexpr bool JM = col_jmaj(N);
    static_assert(MF == 0 || (R0 == 16 && TF % 64 == 0), "matrix-core pass: radix 16, whole waves");
    using F0 = RegPass<N, R0, 1, TF, 1, 0>;
    using F1 = RegPass<N, R1, R0, TF, 1, R0, JM>;
    using F2 = RegPass<N, R2, R0 * R1, TF, 1, 0, JM>;
    using I0 = RegPass<N, R2, 1, TF, 1, 0>;
    using I1 = RegPass<N, R1, R2, TF, 1, R2, JM>;
    using I2 = RegPass<N, R0, R2 * R1, TF, 1, 0, JM>;
    const int tt0 = threadIdx.x, tt = tt0;
    const bool act = tt < TF;
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    int ny = a.ny;
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        W = it.w;
        ny = it.ny;
        a.kh = it.kh;
    }
    // intermediate with C = 2^lc interleaved columns: element i of column v
    // at ((v / C) * ny + i) * C + v % C, the spectrum likewise with ku rows
    const int lc = a.lc, cm = (1 << lc) - 1;
    float2 *const colp = W + ((static_cast<int64_t>(v >> lc) * ny) << lc) + (v & cm);
    // the column's ny stored values through a buffer resource: element n at
    // byte 8 (n << lc), 32-bit offsets from a base held in scalar registers
    const unsigned colb = static_cast<unsigned>((((ny - 1) << lc) + 1) * 8);
    // the result goes to the same place in a.wout (out of place: the stores
    // then never touch lines another column's workgroup still reads)
    const lp_rsrc col = buffer_rsrc(a.wout ? a.wout + (colp - W) : colp, colb);

    // forward transform of one column and product with one spectrum, left in
    // x2 in the order the inverse's first pass takes it
    auto forward = [&](const float2 *srcp, const void *kh, float2 (&x2)[F2::S][R2]) {
        // a class sum re-reads the thread index per call, so that it does not
        // keep per-thread addresses and table offsets live across its class
        // loop
        const int tt = SUM ? opaque_v(tt0) : tt0;
        const lp_rsrc src = buffer_rsrc(srcp, colb);
        float2 x0[F0::S][R0];
        if constexpr (MF != 0) {
            // item i = butterfly i of the column: inputs i + j NB (rows >= ny
            // read as zero), outputs in the layout F0::store writes
            mfma16_items<MF, false, F0::NB, TF / 64, MF_AHEAD_HBM>(
                static_cast<const u4v_t *>(a.mf),
                [&](int i, int j) {
                    const int n = i + j * F0::NB;
                    return bload2(src, static_cast<unsigned>(n << lc) * 8u);  // rows >= ny read zero
                },
                [&](int i, int k, float2 v) { lds[i * lds_pitch(16) + k] = v; });
        } else if (act) {
#pragma unroll
            for (int s = 0; s < F0::S; ++s) {
                const int i = tt + s * TF;
                if (F0::NB % TF == 0 || i < F0::NB) {
#pragma unroll
                    for (int j = 0; j < R0; ++j) {
                        const int n = i + j * F0::NB;
                        // rows >= ny lie past the resource's range: they read zero
                        x0[s][j] = bload2(src, static_cast<unsigned>(n << lc) * 8u);
                    }
                }
            }
            F0::template butterfly<false>(x0, tt);
            F0::store(x0, lds, tt, 0);
        }
        __syncthreads();
        float2 x1[F1::S][R1];
        if (act) {
            F1::load(x1, lds, tt, 0);
            F1::template twiddle<false>(x1, buffer_rsrc(a.tw_f1, F1::TABLE_BYTES), tt);
            F1::template butterfly<false>(x1, tt);
        }
        __syncthreads();
        if (act) F1::store(x1, lds, tt, 0);
        __syncthreads();
        if (act) {
            F2::load(x2, lds, tt, 0);
            F2::template twiddle<false>(x2, buffer_rsrc(a.tw_f2, F2::TABLE_BYTES), tt);
            F2::template butterfly<false>(x2, tt);
            // Eq. 9: pixel-wise product with the kernel spectrum, element u = i + j NB
#pragma unroll
            for (int s = 0; s < F2::S; ++s) {
                const int i = tt + s * TF;
                if (F2::NB % TF == 0 || i < F2::NB) {
                    if constexpr (FORM == 1) {
                        const float *kqp = static_cast<const float *>(kh) +
                                          ((static_cast<int64_t>(v >> lc) * a.ku) << lc) + (v & cm);
                        const lp_rsrc kq = buffer_rsrc(kqp, static_cast<unsigned>((((a.ku - 1) << lc) + 1) * 4));
#pragma unroll
                        for (int j = 0; j < R2; ++j) {
                            const int u = i + j * F2::NB;
                            x2[s][j] = cscale(x2[s][j], bload1(kq, static_cast<unsigned>(((2 * u <= N) ? u : N - u) << lc) * 4u));
                        }
                    } else {
                        const float2 *kcp = static_cast<const float2 *>(kh) +
                                           ((static_cast<int64_t>(v >> lc) * N) << lc) + (v & cm);
                        const lp_rsrc kc = buffer_rsrc(kcp, static_cast<unsigned>((((N - 1) << lc) + 1) * 8));
#pragma unroll
                        for (int j = 0; j < R2; ++j) {
                            const float2 k = bload2(kc, static_cast<unsigned>((i + j * F2::NB) << lc) * 8u);
                            x2[s][j] = CONJ ? cmulc(x2[s][j], k) : cmul(x2[s][j], k);
                        }
                    }
                }
            }
        }
    };

    float2 x2[F2::S][R2];
    forward(colp, a.kh, x2);
    if constexpr (SUM) {
        for (int t = 1; t < a.classes; ++t) {
            float2 z[F2::S][R2];
            __syncthreads();  // every thread is done reading the exchange buffer
            forward(colp + t * a.w_stride, static_cast<const char *>(a.kh) + t * a.kh_stride, z);
            if (act) {
#pragma unroll
                for (int s = 0; s < F2::S; ++s)
#pragma unroll
                    for (int j = 0; j < R2; ++j) x2[s][j] = cadd(x2[s][j], z[s][j]);
            }
        }
    }
    if (act) I0::template butterfly<true>(x2, tt);
    __syncthreads();
    if (act) I0::store(x2, lds, tt, 0);
    __syncthreads();
    float2 y1[I1::S][R1];
    if (act) {
        I1::load(y1, lds, tt, 0);
        I1::template twiddle<true>(y1, buffer_rsrc(a.tw_i1, I1::TABLE_BYTES), tt);
        I1::template butterfly<true>(y1, tt);
    }
    __syncthreads();
    if (act) I1::store(y1, lds, tt, 0);
    __syncthreads();
    if constexpr (MF != 0) {
        // item i = butterfly i: inputs i + j NB of the exchange buffer,
        // twiddled as I2::twiddle does (P = R2 R1 = NB, so i mod P = i);
        // output k is row i + k NB of the column
        constexpr int P = R2 * R1;
        const lp_rsrc tw = buffer_rsrc(a.tw_i2, I2::TABLE_BYTES);
        mfma16_items<MF, true, I2::NB, TF / 64, 1>(
            static_cast<const u4v_t *>(a.mf),
            [&](int i, int j) {
                const float2 v = lds[i + j * I2::NB];
                if (j == 0) return v;
                const unsigned t = JM ? static_cast<unsigned>((j - 1) * P + i) * 8u
                                      : static_cast<unsigned>(i * (R0 - 1) + j - 1) * 8u;
                return cmulc(v, bload2(tw, t));
            },
            [&](int i, int k, float2 v) {
                const int n = i + k * I2::NB;
                bstore2(col, static_cast<unsigned>(n << lc) * 8u, v);  // rows >= ny: dropped
            });
    } else if (act) {
        float2 y2[I2::S][R0];
        I2::load(y2, lds, tt, 0);
        I2::template twiddle<true>(y2, buffer_rsrc(a.tw_i2, I2::TABLE_BYTES), tt);
        I2::template butterfly<true>(y2, tt);
#pragma unroll
        for (int s = 0; s < I2::S; ++s) {
            const int i = tt + s * TF;
            if (I2::NB % TF == 0 || i < I2::NB) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int n = i + j * I2::NB;
                    // rows >= ny lie past the resource's range: the store is dropped
                    bstore2(col, static_cast<unsigned>(n << lc) * 8u, y2[s][j]);
                }
            }
        }
    }
}

// Column kernel with the exchanges in two halves: the same transform,
// product and layouts as k_cols_reg, but each exchange between passes goes
// through a float buffer (same word layout) twice, real parts then imaginary
// parts, so the buffer is half the size and twice as many workgroups fit on
// a CU (2 per CU for 18432-point columns instead of 1).  Each pass's
// arithmetic stays in one divergent block; the register allocator plans for
// exactly OCC waves per SIMD, the occupancy the halved buffer is there to
// reach.
template <class A, class B>
__device__ __forceinline__ void half_mid(const float2 (&x)[A::S][A::RADIX], float2 (&y)[B::S][B::RADIX],
                                         float *f, int tt, bool act)
{
    __syncthreads();
    if (act) B::template load_part<0>(y, f, tt, 0);
    __syncthreads();
    if (act) A::template store_part<1>(x, f, tt, 0);
    __syncthreads();
}

template <int N, int TF, int R0, int R1, int R2, int OCC, int FORM, bool CONJ, bool SUM>
__global__ void __launch_bounds__(((TF + 63) / 64) * 64)
__attribute__((amdgpu_waves_per_eu(SUM ? 0 : OCC, SUM ? 0 : OCC)))
k_cols_half(float2 *__restrict__ W, ColRegArgs a, const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    float *f = reinterpret_cast<float *>(lds);
    constexpr bool JM = col_jmaj(N);
    using F0 = RegPass<N, R0, 1, TF, 1, 0>;
    using F1 = RegPass<N, R1, R0, TF, 1, R0, JM>;
    using F2 = RegPass<N, R2, R0 * R1, TF, 1, 0, JM>;
    using I0 = RegPass<N, R2, 1, TF, 1, 0>;
    using I1 = RegPass<N, R1, R2, TF, 1, R2, JM>;
    using I2 = RegPass<N, R0, R2 * R1, TF, 1, 0, JM>;
    const int tt0 = threadIdx.x, tt = tt0;
    const bool act = tt < TF;
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    int ny = a.ny;
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        W = it.w;
        ny = it.ny;
        a.kh = it.kh;
    }
    const int lc = a.lc, cm = (1 << lc) - 1;
    float2 *const colp = W + ((static_cast<int64_t>(v >> lc) * ny) << lc) + (v & cm);
    // the column's ny stored values through a buffer resource: element n at
    // byte 8 (n << lc), 32-bit offsets from a base held in scalar registers
    const unsigned colb = static_cast<unsigned>((((ny - 1) << lc) + 1) * 8);
    // the result goes to the same place in a.wout (out of place: the stores
    // then never touch lines another column's workgroup still reads)
    const lp_rsrc col = buffer_rsrc(a.wout ? a.wout + (colp - W) : colp, colb);

    // Eq. 9: product of the last forward pass's outputs (element u = i + j NB)
    // with the kernel spectrum
    auto multiply = [&](float2 (&xl)[F2::S][R2], const void *kh, int tt) {
#pragma unroll
        for (int s = 0; s < F2::S; ++s) {
            const int i = tt + s * TF;
            if (F2::valid(i)) {
                if constexpr (FORM == 1) {
                    const float *kqp = static_cast<const float *>(kh) +
                                      ((static_cast<int64_t>(v >> lc) * a.ku) << lc) + (v & cm);
                    const lp_rsrc kq = buffer_rsrc(kqp, static_cast<unsigned>((((a.ku - 1) << lc) + 1) * 4));
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int u = i + j * F2::NB;
                        xl[s][j] = cscale(xl[s][j], bload1(kq, static_cast<unsigned>(((2 * u <= N) ? u : N - u) << lc) * 4u));
                    }
                } else {
                    const float2 *kcp = static_cast<const float2 *>(kh) +
                                       ((static_cast<int64_t>(v >> lc) * N) << lc) + (v & cm);
                    const lp_rsrc kc = buffer_rsrc(kcp, static_cast<unsigned>((((N - 1) << lc) + 1) * 8));
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const float2 k = bload2(kc, static_cast<unsigned>((i + j * F2::NB) << lc) * 8u);
                        xl[s][j] = CONJ ? cmulc(xl[s][j], k) : cmul(xl[s][j], k);
                    }
                }
            }
        }
    };

    auto forward = [&](const float2 *srcp, const void *kh, float2 (&xl)[F2::S][R2]) {
        // a class sum re-reads the thread index per call, so that it does not
        // keep per-thread addresses and table offsets live across its class
        // loop
        const int tt = SUM ? opaque_v(tt0) : tt0;
        const lp_rsrc src = buffer_rsrc(srcp, colb);
        float2 x0[F0::S][R0];
        if (act) {
#pragma unroll
            for (int s = 0; s < F0::S; ++s) {
                const int i = tt + s * TF;
                if (F0::valid(i)) {
#pragma unroll
                    for (int j = 0; j < R0; ++j) {
                        const int n = i + j * F0::NB;
                        // rows >= ny lie past the resource's range: they read zero
                        x0[s][j] = bload2(src, static_cast<unsigned>(n << lc) * 8u);
                    }
                }
            }
            F0::template butterfly<false>(x0, tt);
            F0::template store_part<0>(x0, f, tt, 0);
        }
        float2 x1[F1::S][R1];
        half_mid<F0, F1>(x0, x1, f, tt, act);
        if (act) {
            F1::template load_part<1>(x1, f, tt, 0);
            F1::template twiddle<false>(x1, buffer_rsrc(a.tw_f1, F1::TABLE_BYTES), tt);
            F1::template butterfly<false>(x1, tt);
        }
        __syncthreads();
        if (act) F1::template store_part<0>(x1, f, tt, 0);
        half_mid<F1, F2>(x1, xl, f, tt, act);
        if (act) {
            F2::template load_part<1>(xl, f, tt, 0);
            F2::template twiddle<false>(xl, buffer_rsrc(a.tw_f2, F2::TABLE_BYTES), tt);
            F2::template butterfly<false>(xl, tt);
            multiply(xl, kh, tt);
        }
    };

    // the last inverse pass writes rows < ny of the column
    auto store_out = [&](const float2 (&y)[I2::S][R0]) {
#pragma unroll
        for (int s = 0; s < I2::S; ++s) {
            const int i = tt + s * TF;
            if (I2::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int n = i + j * I2::NB;
                    // rows >= ny lie past the resource's range: the store is dropped
                    bstore2(col, static_cast<unsigned>(n << lc) * 8u, y[s][j]);
                }
            }
        }
    };

    float2 xl[F2::S][R2];
    forward(colp, a.kh, xl);
    if constexpr (SUM) {
        for (int t = 1; t < a.classes; ++t) {
            float2 z[F2::S][R2];
            __syncthreads();  // every thread is done reading the exchange buffer
            forward(colp + t * a.w_stride, static_cast<const char *>(a.kh) + t * a.kh_stride, z);
            if (act) {
#pragma unroll
                for (int s = 0; s < F2::S; ++s)
#pragma unroll
                    for (int j = 0; j < R2; ++j) xl[s][j] = cadd(xl[s][j], z[s][j]);
            }
        }
    }
    if (act) I0::template butterfly<true>(xl, tt);
    __syncthreads();
    if (act) I0::template store_part<0>(xl, f, tt, 0);
    float2 y1[I1::S][R1];
    half_mid<I0, I1>(xl, y1, f, tt, act);
    if (act) {
        I1::template load_part<1>(y1, f, tt, 0);
        I1::template twiddle<true>(y1, buffer_rsrc(a.tw_i1, I1::TABLE_BYTES), tt);
        I1::template butterfly<true>(y1, tt);
    }
    __syncthreads();
    if (act) I1::template store_part<0>(y1, f, tt, 0);
    float2 y2[I2::S][R0];
    half_mid<I1, I2>(y1, y2, f, tt, act);
    if (act) {
        I2::template load_part<1>(y2, f, tt, 0);
        I2::template twiddle<true>(y2, buffer_rsrc(a.tw_i2, I2::TABLE_BYTES), tt);
        I2::template butterfly<true>(y2, tt);
        store_out(y2);
    }
}

int col_spec_index(int n, int k)
{
    for (int i = 0; i < kNumColSpecs; ++i)
        if (kColSpecs[i].n == n && k-- == 0) return i;
    return -1;
}

int col_spec_count(int n)
{
    int c = 0;
    for (int i = 0; i < kNumColSpecs; ++i) c += kColSpecs[i].n == n;
    return c;
}

static constexpr int xchg_words(int n, int r0, int r2)
{
    const int a = lds_words(n, r0), c = lds_words(n, r2);
    const int m = a > c ? a : c;
    return m > n ? m : n;
}

// Middle kernel of the four-step column stage with register-resident
// transforms, for a split whose P2 has a specialisation: workgroup (v, k1)
// takes the P2 values T[v][k1][.] (contiguous), transforms them with the
// passes of k_cols_reg (radices R0, R1, R2), multiplies by the spectrum at
// stored rows k1 P2 + k2 (the four-step order, contiguous), transforms back
// and multiplies by exp(+2 pi i n2 k1 / Py), in place.  Tables: c.tw_* for
// length P2; a.twq for the four-step twiddles.
template <int N, int TF, int R0, int R1, int R2, int OCC, int FORM, bool CONJ>
__global__ void __launch_bounds__(((TF + 63) / 64) * 64, OCC) k_long_mid_reg(LongArgs a, ColRegArgs c)
{
    extern __shared__ float2 lds[];
    constexpr bool JM = col_jmaj(N);
    using F0 = RegPass<N, R0, 1, TF, 1, 0>;
    using F1 = RegPass<N, R1, R0, TF, 1, R0, JM>;
    using F2 = RegPass<N, R2, R0 * R1, TF, 1, 0, JM>;
    using I0 = RegPass<N, R2, 1, TF, 1, 0>;
    using I1 = RegPass<N, R1, R2, TF, 1, R2, JM>;
    using I2 = RegPass<N, R0, R2 * R1, TF, 1, 0, JM>;
    const int tt = threadIdx.x;
    const bool act = tt < TF;
    // the two columns of an interleaved group on one XCD (shared spectrum lines)
    const int v = xcd_tile(blockIdx.x, gridDim.x), k1 = blockIdx.y;
    float2 *t = a.T + static_cast<int64_t>(v) * a.py + static_cast<int64_t>(k1) * N;
    float2 x0[F0::S][R0];
    if (act) {
#pragma unroll
        for (int s = 0; s < F0::S; ++s) {
            const int i = tt + s * TF;
            if (F0::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) x0[s][j] = t[i + j * F0::NB];
            }
        }
        F0::template butterfly<false>(x0, tt);
        F0::store(x0, lds, tt, 0);
    }
    __syncthreads();
    float2 x1[F1::S][R1];
    if (act) {
        F1::load(x1, lds, tt, 0);
        F1::template twiddle<false>(x1, c.tw_f1, tt);
        F1::template butterfly<false>(x1, tt);
    }
    __syncthreads();
    if (act) F1::store(x1, lds, tt, 0);
    __syncthreads();
    float2 x2[F2::S][R2];
    if (act) {
        F2::load(x2, lds, tt, 0);
        F2::template twiddle<false>(x2, c.tw_f2, tt);
        F2::template butterfly<false>(x2, tt);
        // Eq. 9: frequency k1 + P1 k2 with k2 = u = i + j NB, stored row k1 P2 + k2
        const int lc = a.lc, cm = (1 << lc) - 1;
        const int64_t base = ((static_cast<int64_t>(v >> lc) * a.py + static_cast<int64_t>(k1) * N) << lc) + (v & cm);
#pragma unroll
        for (int s = 0; s < F2::S; ++s) {
            const int i = tt + s * TF;
            if (F2::valid(i)) {
#pragma unroll
                for (int j = 0; j < R2; ++j) {
                    const int64_t idx = base + (static_cast<int64_t>(i + j * F2::NB) << lc);
                    if constexpr (FORM == 1) {
                        x2[s][j] = cscale(x2[s][j], static_cast<const float *>(a.kh)[idx]);
                    } else {
                        const float2 k = static_cast<const float2 *>(a.kh)[idx];
                        x2[s][j] = CONJ ? cmulc(x2[s][j], k) : cmul(x2[s][j], k);
                    }
                }
            }
        }
        I0::template butterfly<true>(x2, tt);
    }
    __syncthreads();
    if (act) I0::store(x2, lds, tt, 0);
    __syncthreads();
    float2 y1[I1::S][R1];
    if (act) {
        I1::load(y1, lds, tt, 0);
        I1::template twiddle<true>(y1, c.tw_i1, tt);
        I1::template butterfly<true>(y1, tt);
    }
    __syncthreads();
    if (act) I1::store(y1, lds, tt, 0);
    __syncthreads();
    if (act) {
        float2 y2[I2::S][R0];
        I2::load(y2, lds, tt, 0);
        I2::template twiddle<true>(y2, c.tw_i2, tt);
        I2::template butterfly<true>(y2, tt);
#pragma unroll
        for (int s = 0; s < I2::S; ++s) {
            const int i = tt + s * TF;
            if (I2::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int n = i + j * I2::NB;
                    // n k1 < P2 P1 = Py: no reduction needed
                    t[n] = cmulc(y2[s][j], a.twq[n * k1]);
                }
            }
        }
    }
}

// The specialisation the four-step middle kernel uses for a length: the
// first full-exchange column variant of that length (-1: none).
// the four-step middle transforms run FP32 register kernels: the first
// full-exchange FP32 specialisation of the length
int long_mid_spec(int n)
{
    for (int i = 0; i < kNumColSpecs; ++i)
        if (kColSpecs[i].n == n && !kColSpecs[i].half && !kColSpecs[i].mf) return i;
    return -1;
}

static constexpr bool is_long_mid_spec(int I)
{
    for (int i = 0; i < I; ++i)
        if (kColSpecs[i].n == kColSpecs[I].n && !kColSpecs[i].half && !kColSpecs[i].mf) return false;
    return !kColSpecs[I].half && !kColSpecs[I].mf;
}

template <int I>
static hipError_t long_mid_from(int idx, const LongArgs &a, const ColRegArgs &c, int ncols, int form,
                                bool conj_k, hipStream_t s, bool attrs_only)
{
    if constexpr (I >= kNumColSpecs) {
        return attrs_only ? hipSuccess : hipErrorInvalidValue;
    } else if constexpr (!is_long_mid_spec(I)) {
        return long_mid_from<I + 1>(idx, a, c, ncols, form, conj_k, s, attrs_only);
    } else {
        constexpr ColSpec cs = kColSpecs[I];
        constexpr size_t lds = static_cast<size_t>(xchg_words(cs.n, cs.r0, cs.r2)) * 8;
        if (attrs_only) {
            const void *fns[] = {
                reinterpret_cast<const void *>(&k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 1, false>),
                reinterpret_cast<const void *>(&k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 2, false>),
                reinterpret_cast<const void *>(&k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 2, true>)};
            for (const void *f : fns) {
                hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
                if (e != hipSuccess) return e;
            }
            return long_mid_from<I + 1>(idx, a, c, ncols, form, conj_k, s, attrs_only);
        }
        if (idx != I) return long_mid_from<I + 1>(idx, a, c, ncols, form, conj_k, s, attrs_only);
        if (a.p2 != cs.n) return hipErrorInvalidValue;
        const dim3 g(ncols, a.p1), t(((cs.tf + 63) / 64) * 64);
        if (form == 1)
            hipLaunchKernelGGL((k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 1, false>), g, t, lds, s, a, c);
        else if (conj_k)
            hipLaunchKernelGGL((k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 2, true>), g, t, lds, s, a, c);
        else
            hipLaunchKernelGGL((k_long_mid_reg<cs.n, cs.tf, cs.r0, cs.r1, cs.r2, cs.occ, 2, false>), g, t, lds, s, a, c);
        return hipGetLastError();
    }
}

hipError_t launch_long_mid_reg(const LongArgs &a, const ColRegArgs &c, int idx, int ncols, int form, bool conj_k,
                               hipStream_t s)
{
    return long_mid_from<0>(idx, a, c, ncols, form, conj_k, s, false);
}

hipError_t set_long_mid_attributes()
{
    LongArgs a{};
    ColRegArgs c{};
    return long_mid_from<0>(-1, a, c, 0, 1, false, nullptr, true);
}


template <int I>
static constexpr size_t col_lds_bytes()
{
    return static_cast<size_t>(xchg_words(kColSpecs[I].n, kColSpecs[I].r0, kColSpecs[I].r2)) * (kColSpecs[I].half ? 4 : 8);
}

// SPLIT: the split form of a variant with a matrix-core pass (1 or 2; 0 for
// the other variants)
template <int I, int FORM, bool CONJ, bool SUM = false, int SPLIT = (kColSpecs[I].mf ? 2 : 0)>
static const void *col_fn()
{
    constexpr ColSpec c = kColSpecs[I];
    static_assert(!c.mf || !c.half, "matrix-core columns: full exchange");
    static_assert((SPLIT != 0) == (c.mf != 0), "split form of a matrix-core variant");
    if constexpr (c.half)
        return reinterpret_cast<const void *>(&k_cols_half<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM>);
    else
        return reinterpret_cast<const void *>(&k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM, SPLIT>);
}

template <int I, int FORM, bool CONJ, bool SUM>
static void launch_col(dim3 g, dim3 t, size_t lds, hipStream_t s, float2 *W, const ColRegArgs &a,
                       const BatchItem *items)
{
    constexpr ColSpec c = kColSpecs[I];
    if constexpr (c.half)
        hipLaunchKernelGGL((k_cols_half<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM>), g, t, lds, s, W, a, items);
    else if constexpr (c.mf) {
        if (a.split == 1)
            hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM, 1>), g, t, lds, s, W, a, items);
        else
            hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM, 2>), g, t, lds, s, W, a, items);
    } else
        hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, c.occ, FORM, CONJ, SUM>), g, t, lds, s, W, a, items);
}

template <int I>
static hipError_t col_attrs_from()
{
    if constexpr (I >= kNumColSpecs) {
        return hipSuccess;
    } else {
        constexpr int NS = kColSpecs[I].mf ? 2 : 1;  // instances per form
        const void *fns[5 * NS];
        if constexpr (kColSpecs[I].mf) {
            const void *t[10] = {col_fn<I, 1, false, false, 1>(), col_fn<I, 2, false, false, 1>(),
                                 col_fn<I, 2, true, false, 1>(), col_fn<I, 1, false, true, 1>(),
                                 col_fn<I, 2, false, true, 1>(), col_fn<I, 1, false, false, 2>(),
                                 col_fn<I, 2, false, false, 2>(), col_fn<I, 2, true, false, 2>(),
                                 col_fn<I, 1, false, true, 2>(), col_fn<I, 2, false, true, 2>()};
            std::copy(t, t + 10, fns);
        } else {
            const void *t[5] = {col_fn<I, 1, false>(), col_fn<I, 2, false>(), col_fn<I, 2, true>(),
                                col_fn<I, 1, false, true>(), col_fn<I, 2, false, true>()};
            std::copy(t, t + 5, fns);
        }
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
            if (e != hipSuccess) return e;
        }
        return col_attrs_from<I + 1>();
    }
}

template <int I>
static hipError_t launch_col_from(int idx, float2 *W, const ColRegArgs &a, int ncols, int form,
                                  bool conj_k, hipStream_t s, const BatchItem *items, int nitems,
                                  bool sum)
{
    if constexpr (I >= kNumColSpecs) {
        return hipErrorInvalidValue;
    } else {
        if (idx != I) return launch_col_from<I + 1>(idx, W, a, ncols, form, conj_k, s, items, nitems, sum);
        constexpr ColSpec c = kColSpecs[I];
        const dim3 g(ncols, nitems), t(((c.tf + 63) / 64) * 64);
        const size_t lds = col_lds_bytes<I>();
        if (sum && conj_k) return hipErrorInvalidValue;  // class sums are forward only
        // a matrix-core variant needs its split form and fragment table
        if (c.mf && (!a.mf || (a.split != 1 && a.split != 2))) return hipErrorInvalidValue;
        const ColRegArgs &b = a;
        if (sum && form == 1)
            launch_col<I, 1, false, true>(g, t, lds, s, W, b, items);
        else if (sum)
            launch_col<I, 2, false, true>(g, t, lds, s, W, b, items);
        else if (form == 1)
            launch_col<I, 1, false, false>(g, t, lds, s, W, b, items);
        else if (conj_k)
            launch_col<I, 2, true, false>(g, t, lds, s, W, b, items);
        else
            launch_col<I, 2, false, false>(g, t, lds, s, W, b, items);
        return hipGetLastError();
    }
}

hipError_t launch_cols_reg(float2 *W, const ColRegArgs &a, int idx, int ncols, int form, bool conj_k,
                           hipStream_t s, const BatchItem *items, int nitems, bool class_sum)
{
    hipError_t e = set_spec_attributes();
    if (e != hipSuccess) return e;
    return launch_col_from<0>(idx, W, a, ncols, form, conj_k, s, items, nitems, class_sum);
}

}  // namespace lp

// ======================================================= register-resident rows
namespace lp {

typedef float lp_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void gstore4(gptr<float2> p, float2 a, float2 b)
{
    const lp_f4v v = {a.x, a.y, b.x, b.y};
    *(gptr<lp_f4v>)p = v;
}
__device__ __forceinline__ void gload4(gptr<const float2> p, float2 &a, float2 &b)
{
    const lp_f4v v = *(gptr<const lp_f4v>)p;
    a = make_float2(v.x, v.y);
    b = make_float2(v.z, v.w);
}

// Staged intermediate of B consecutive rows (row0 = tile * B, B even or 1):
// spectrum column k of row row0 + b at lds[k * B + b], 0 <= k <= M + 1 (the
// last column is the pad of the two-column interleave when M + 1 is odd).
// In HBM the pair of columns (2p, 2p + 1) of rows row0 .. row0 + B - 1 is one
// run of 16 B bytes: chunk c = p B + b is row b's 16 bytes at
// ((p ny + row0 + b) << 1).
template <int M, int B>
struct RowStage {
    static constexpr int NCHUNK = ((M + 2) / 2) * B;
    template <int NT>
    static constexpr int per_thread() { return (NCHUNK + NT - 1) / NT; }
};

// Row z[n] = x[2n] + i x[2n+1] of the zero-padded map (columns >= nx, rows
// >= ny are zero).
template <bool EVEN_NX>
__device__ __forceinline__ float2 load_pair(gptr<const float> src, int n, int nx, bool rv)
{
    const int c0 = 2 * n;
    if (!rv || c0 >= nx) return make_float2(0.f, 0.f);
    if (EVEN_NX) return gload2_nt(src + c0);  // read once: a streaming load
    return make_float2(src[c0], (c0 + 1 < nx) ? src[c0 + 1] : 0.f);
}

// X[k] = E + w^k O from Z[k] (z) and Z[M-k] (zp): E = (z + conj zp)/2,
// O = -i (z - conj zp)/2.
__device__ __forceinline__ float2 r2c_split(float2 z, float2 zp, float2 w)
{
    const float2 E = make_float2(0.5f * (z.x + zp.x), 0.5f * (z.y - zp.y));
    const float2 O = make_float2(0.5f * (z.y + zp.y), -0.5f * (z.x - zp.x));
    return cadd(E, cmul(O, w));
}

// Twice the spectrum of x[2n] + i x[2n+1] at k from X[k] (x) and X[M-k] (xp):
// (x + conj xp) + i conj(w^k) (x - conj xp).
__device__ __forceinline__ float2 c2r_merge(float2 x, float2 xp, float2 w)
{
    const float2 s = make_float2(x.x + xp.x, x.y - xp.y);
    const float2 d = make_float2(x.x - xp.x, x.y + xp.y);
    const float2 wd = cmulc(d, w);
    return make_float2(s.x - wd.y, s.y + wd.x);
}

// Forward rows.  Passes R0, R1 in the usual thread mapping; the last pass
// (radix R2, NB = M/R2 butterflies) gives thread tt the butterflies tt and
// NB - tt, so that it holds both Z[k] and Z[M-k] for every k it produced and
// the real-to-complex split happens in registers.  Output in the column
// interleave C = 2^lc: X[k] of row r at ((k / C) ny + r) C + k mod C (STG:
// through LDS, in 16-byte chunks of a column pair).  MF (1 or 2): the
// radix-16 first pass (R0 = 16) runs on the matrix cores in that split form,
// reading the rows straight from HBM.
// TPW tiles of B rows per workgroup, g and g + G (G = grid size); with two,
// the second tile's inputs are loaded into registers before the first is
// transformed, so its HBM reads overlap the arithmetic.  The code is straight
// line (no loop) so that the DFT constants are not hoisted into registers
// that stay live across iterations.
template <int M, int TF, int R0, int R1, int R2, int B, int OCC, int TPW, bool EVEN_NX, bool STG = false, int MF = 0>
__global__ void __launch_bounds__(TF * B, OCC) k_rows_r2c_reg(const float *__restrict__ Rm,
                                                             float2 *__restrict__ W, RowRegArgs a,
                                                             const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    using F0 = RegPass<M, R0, 1, TF, B, 0>;
    using F1 = RegPass<M, R1, R0, TF, B, R0>;
    constexpr int NB = M / R2;
    static_assert(R0 * R1 * R2 == M && NB / 2 + 1 <= TF, "row specialisation");
    static_assert(TPW >= 0 && TPW <= 2, "tiles per workgroup");
    static_assert(!STG || TPW == 1, "staged rows take one tile per workgroup");
    static_assert(MF == 0 || (R0 == 16 && TPW == 1 && (TF * B) % 64 == 0),
                  "matrix-core first pass: radix 16, one tile per workgroup, whole waves");
    const int tid0 = threadIdx.x;
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        Rm = it.in;
        W = it.w;
        a.ny = it.ny;
        a.nx = it.nx;
    }
    const int ntiles = (a.ny + B - 1) / B;
    const int G = gridDim.x;
    const int64_t ny = a.ny;

    auto load_tile = [&](float2 (&x)[F0::S][R0], int tile, int tt, int b) {
        const int row = tile * B + b;
        const bool rv = row < a.ny;
        const gptr<const float> src = as_global(Rm) + static_cast<int64_t>(rv ? row : 0) * a.nx;
#pragma unroll
        for (int s = 0; s < F0::S; ++s) {
            const int i = tt + s * TF;
            if (F0::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) x[s][j] = load_pair<EVEN_NX>(src, i + j * F0::NB, a.nx, rv);
            }
        }
    };

    auto transform = [&](float2 (&x0)[F0::S][R0], int tile, int tt, int b) {
        const int row = tile * B + b;
        const bool rv = row < a.ny;
        if constexpr (MF != 0) {
            // the radix-16 first pass on the matrix cores, straight from HBM:
            // item w = (row tile*B + w / F0::NB, butterfly w % F0::NB), its
            // outputs in the layout F0::store writes
            const gptr<const float> src = as_global(Rm);
            mfma16_items<MF, false, F0::NB * B, TF * B / 64, MF_AHEAD_HBM>(
                static_cast<const u4v_t *>(a.mf),
                [&](int w, int j) {
                    const int bb = w / F0::NB, i = w % F0::NB, r = tile * B + bb;
                    const bool ok = r < a.ny;
                    return load_pair<EVEN_NX>(src + static_cast<int64_t>(ok ? r : 0) * a.nx, i + j * F0::NB, a.nx, ok);
                },
                [&](int w, int k, float2 v) {
                    const int bb = w / F0::NB, i = w % F0::NB;
                    lds[(i * lds_pitch(16) + k) * B + bb] = v;
                });
        } else {
            F0::template butterfly<false>(x0, tt);
            F0::store(x0, lds, tt, b);
        }
        __syncthreads();
        {
            float2 x1[F1::S][R1];
            F1::load(x1, lds, tt, b);
            F1::template twiddle<false>(x1, a.tw_f1, tt);
            F1::template butterfly<false>(x1, tt);
            __syncthreads();
            F1::store(x1, lds, tt, b);
        }
        __syncthreads();
        const int i1 = tt, i2 = NB - tt;
        const bool pairer = tt <= NB / 2;
        const bool two = pairer && (i2 != i1) && (i2 < NB);
        float2 z1[R2], z2[R2];
        if (pairer) {
#pragma unroll
            for (int j = 0; j < R2; ++j) z1[j] = lds[(i1 + j * NB) * B + b];
            if (i1 > 0) {
#pragma unroll
                for (int j = 1; j < R2; ++j) z1[j] = cmul(z1[j], a.tw_f2[i1 * (R2 - 1) + j - 1]);
            }
            dftc<R2, false>(z1);
            if (two) {
#pragma unroll
                for (int j = 0; j < R2; ++j) z2[j] = lds[(i2 + j * NB) * B + b];
#pragma unroll
                for (int j = 1; j < R2; ++j) z2[j] = cmul(z2[j], a.tw_f2[i2 * (R2 - 1) + j - 1]);
                dftc<R2, false>(z2);
            }
        }
        if constexpr (STG) {
            // spectrum X[k] of the tile's rows into the exchange buffer (every
            // thread has read its last-pass inputs), then out in 16-byte chunks
            __syncthreads();
            if (pairer) {
                if (i1 == 0) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k = j * NB;
                        lds[k * B + b] = r2c_split(z1[j], z1[(R2 - j) % R2], a.rtw[k]);
                    }
                    lds[M * B + b] = r2c_split(z1[0], z1[0], a.rtw[M]);
                    lds[(M + 1) * B + b] = make_float2(0.f, 0.f);
                } else if (!two) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k = i1 + j * NB;
                        lds[k * B + b] = r2c_split(z1[j], z1[R2 - 1 - j], a.rtw[k]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k1 = i1 + j * NB, k2 = i2 + j * NB;
                        lds[k1 * B + b] = r2c_split(z1[j], z2[R2 - 1 - j], a.rtw[k1]);
                        lds[k2 * B + b] = r2c_split(z2[j], z1[R2 - 1 - j], a.rtw[k2]);
                    }
                }
            }
            __syncthreads();
            using ST = RowStage<M, B>;
            constexpr int NT = TF * B, PT = ST::template per_thread<NT>();
            const int tid = tt * B + b;
            const gptr<float2> dst = as_global(W) + (static_cast<int64_t>(tile * B) << 1);
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                const int c = tid + q * NT;
                const int p = c / B, bb = c % B;
                if ((ST::NCHUNK % NT == 0 || c < ST::NCHUNK) && tile * B + bb < a.ny)
                    gstore4(dst + ((static_cast<int64_t>(p) * ny + bb) << 1), lds[(2 * p) * B + bb],
                            lds[(2 * p + 1) * B + bb]);
            }
        } else if (pairer && rv) {
            {
                // X[k] of this row at ((k / C) * ny + row) * C + k % C
                const int lc = a.lc, cm = (1 << lc) - 1;
                const gptr<float2> dst = as_global(W) + (static_cast<int64_t>(row) << lc);
                auto at = [&](int k) { return ((static_cast<int64_t>(k >> lc) * ny) << lc) + (k & cm); };
                if (i1 == 0) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k = j * NB;
                        gstore2(dst + at(k), r2c_split(z1[j], z1[(R2 - j) % R2], a.rtw[k]));
                    }
                    gstore2(dst + at(M), r2c_split(z1[0], z1[0], a.rtw[M]));
                } else if (!two) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k = i1 + j * NB;
                        gstore2(dst + at(k), r2c_split(z1[j], z1[R2 - 1 - j], a.rtw[k]));
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int k1 = i1 + j * NB, k2 = i2 + j * NB;
                        gstore2(dst + at(k1), r2c_split(z1[j], z2[R2 - 1 - j], a.rtw[k1]));
                        gstore2(dst + at(k2), r2c_split(z2[j], z1[R2 - 1 - j], a.rtw[k2]));
                    }
                }
            }
        }
    };

    // one tile per workgroup: the item's own tiles are dealt out (in a batch
    // the grid spans the largest item)
    const int t0 = (TPW == 1) ? kept_tile(blockIdx.x, ntiles, B, 0, a.ny) : xcd_tile(blockIdx.x, G);
    if (t0 < 0 || t0 >= ntiles) return;
    const int tt0 = tid0 / B, b0 = tid0 % B;
    if constexpr (TPW == 1) {
        float2 x0[F0::S][R0];
        if constexpr (MF == 0) load_tile(x0, t0, tt0, b0);
        transform(x0, t0, tt0, b0);
    } else if constexpr (TPW == 2) {
        const int t1 = t0 + G;
        float2 x0[F0::S][R0], xn[F0::S][R0];
        load_tile(x0, t0, tt0, b0);
        if (t1 < ntiles) load_tile(xn, t1, tt0, b0);
        transform(x0, t0, tt0, b0);
        if (t1 < ntiles) {
            __syncthreads();  // the second tile's first pass rewrites the exchange buffer
            transform(xn, t1, tt0, b0);
        }
    } else {
        // Persistent: tiles t0, t0 + G, ... with the next tile prefetched.  The
        // thread index is re-read through opaque_v each iteration so that
        // address arithmetic is not hoisted into loop-long registers.
        float2 xn[F0::S][R0];
        load_tile(xn, t0, tt0, b0);
        for (int t = t0; t < ntiles; t += G) {
            const int tid = opaque_v(tid0), tt = tid / B, b = tid % B;
            float2 x0[F0::S][R0];
#pragma unroll
            for (int s = 0; s < F0::S; ++s)
#pragma unroll
                for (int j = 0; j < R0; ++j) x0[s][j] = xn[s][j];
            if (t + G < ntiles) load_tile(xn, t + G, tt, b);
            transform(x0, t, tt, b);
            __syncthreads();
        }
    }
}

// Inverse rows: the first pass (radix R2, NB = M/R2) pairs butterflies tt and
// NB - tt so that X[k] and X[M-k] are merged in registers; then passes R1
// and R0; row outputs x[2n], x[2n+1] for columns < nx (the crop).  TPW tiles
// per workgroup as in the forward kernel.  MF (1 or 2): the radix-16 last
// pass (R0 = 16) runs on the matrix cores in that split form and writes the
// rows straight to HBM.
template <int M, int TF, int R0, int R1, int R2, int B, int OCC, int TPW, bool EVEN_NX, bool STG = false, int MF = 0>
__global__ void __launch_bounds__(TF * B, OCC) k_rows_c2r_reg(const float2 *__restrict__ W,
                                                             float *__restrict__ Sm, RowRegArgs a,
                                                             const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    using I1 = RegPass<M, R1, R2, TF, B, R2>;
    using I2 = RegPass<M, R0, R2 * R1, TF, B, 0>;
    constexpr int NB = M / R2;
    static_assert(R0 * R1 * R2 == M && NB / 2 + 1 <= TF, "row specialisation");
    static_assert(TPW >= 0 && TPW <= 2, "tiles per workgroup");
    static_assert(!STG || TPW == 1, "staged rows take one tile per workgroup");
    static_assert(MF == 0 || (R0 == 16 && TPW == 1 && (TF * B) % 64 == 0),
                  "matrix-core last pass: radix 16, one tile per workgroup, whole waves");
    const int tid0 = threadIdx.x;
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        W = it.w;
        Sm = it.out;
        a.ny = it.ny;
        a.nx = it.nx;
        a.keep0 = it.keep0;
        a.keep1 = it.keep1;
    }
    const int ntiles = (a.ny + B - 1) / B;
    const int G = gridDim.x;
    const int64_t ny = a.ny;

    auto load_tile = [&](float2 (&xa)[R2], float2 (&xb)[R2], float2 &xm, int tile, int tt, int b) {
        const bool pairer = tt <= NB / 2;
        const int i1 = tt, i2 = NB - tt;
        const bool two = pairer && (i2 != i1) && (i2 < NB);
        const int row = tile * B + b;
        const bool rv = row >= a.keep0 && row < a.keep1;  // rows outside are not needed
        // X[k] of this row at ((k / C) * ny + row) * C + k % C
        const int lc = a.lc, cm = (1 << lc) - 1;
        const gptr<const float2> src = as_global(W) + (static_cast<int64_t>(rv ? row : 0) << lc);
        auto at = [&](int k) { return ((static_cast<int64_t>(k >> lc) * ny) << lc) + (k & cm); };
#pragma unroll
        for (int j = 0; j < R2; ++j) {
            xa[j] = make_float2(0.f, 0.f);
            xb[j] = make_float2(0.f, 0.f);
        }
        xm = make_float2(0.f, 0.f);
        if (rv && pairer) {
            if constexpr (STG) {
                // from the staged tile (stage_in, then a barrier)
#pragma unroll
                for (int j = 0; j < R2; ++j) xa[j] = lds[(i1 + j * NB) * B + b];
                if (two) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) xb[j] = lds[(i2 + j * NB) * B + b];
                }
                if (i1 == 0) xm = lds[M * B + b];
            } else {
#pragma unroll
                for (int j = 0; j < R2; ++j) xa[j] = gload2(src + at(i1 + j * NB));
                if (two) {
#pragma unroll
                    for (int j = 0; j < R2; ++j) xb[j] = gload2(src + at(i2 + j * NB));
                }
                if (i1 == 0) xm = gload2(src + at(M));
            }
        }
    };

    // The tile's spectrum from HBM into the exchange buffer in 16-byte chunks
    // (kept rows only); every chunk is loaded before any is written.
    auto stage_in = [&](int tile) {
        using ST = RowStage<M, B>;
        constexpr int NT = TF * B, PT = ST::template per_thread<NT>();
        const int tid = threadIdx.x;
        const gptr<const float2> src = as_global(W) + (static_cast<int64_t>(tile * B) << 1);
        float2 v0[PT], v1[PT];
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int c = tid + q * NT;
            const int p = c / B, bb = c % B, row = tile * B + bb;
            v0[q] = v1[q] = make_float2(0.f, 0.f);
            if ((ST::NCHUNK % NT == 0 || c < ST::NCHUNK) && row >= a.keep0 && row < a.keep1)
                gload4(src + ((static_cast<int64_t>(p) * ny + bb) << 1), v0[q], v1[q]);
        }
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int c = tid + q * NT;
            const int p = c / B, bb = c % B;
            if (ST::NCHUNK % NT == 0 || c < ST::NCHUNK) {
                lds[(2 * p) * B + bb] = v0[q];
                lds[(2 * p + 1) * B + bb] = v1[q];
            }
        }
    };

    auto transform = [&](float2 (&xa)[R2], float2 (&xb)[R2], float2 xm, int tile, int tt, int b) {
        const bool pairer = tt <= NB / 2;
        const int i1 = tt, i2 = NB - tt;
        const bool two = pairer && (i2 != i1) && (i2 < NB);
        const int row = tile * B + b;
        const bool rv = row >= a.keep0 && row < a.keep1;  // rows outside are not needed
        if (pairer) {
            float2 za[R2], zb[R2];
            if (i1 == 0) {
#pragma unroll
                for (int j = 0; j < R2; ++j) za[j] = c2r_merge(xa[j], j ? xa[(R2 - j) % R2] : xm, a.rtw[j * NB]);
            } else if (!two) {
#pragma unroll
                for (int j = 0; j < R2; ++j) za[j] = c2r_merge(xa[j], xa[R2 - 1 - j], a.rtw[i1 + j * NB]);
            } else {
#pragma unroll
                for (int j = 0; j < R2; ++j) {
                    za[j] = c2r_merge(xa[j], xb[R2 - 1 - j], a.rtw[i1 + j * NB]);
                    zb[j] = c2r_merge(xb[j], xa[R2 - 1 - j], a.rtw[i2 + j * NB]);
                }
            }
            dftc<R2, true>(za);
#pragma unroll
            for (int j = 0; j < R2; ++j) lds[(i1 * lds_pitch(R2) + j) * B + b] = za[j];
            if (two) {
                dftc<R2, true>(zb);
#pragma unroll
                for (int j = 0; j < R2; ++j) lds[(i2 * lds_pitch(R2) + j) * B + b] = zb[j];
            }
        }
        __syncthreads();
        {
            float2 y1[I1::S][R1];
            I1::load(y1, lds, tt, b);
            I1::template twiddle<true>(y1, a.tw_i1, tt);
            I1::template butterfly<true>(y1, tt);
            __syncthreads();
            I1::store(y1, lds, tt, b);
        }
        __syncthreads();
        if constexpr (MF != 0) {
            // the radix-16 last pass on the matrix cores: item w = (row
            // tile*B + w / I2::NB, butterfly i = w % I2::NB); output k is
            // element i + k I2::NB of the row, written to HBM (the crop)
            mfma16_items<MF, true, I2::NB * B, TF * B / 64, 1>(
                static_cast<const u4v_t *>(a.mf),
                [&](int w, int j) {
                    const int bb = w / I2::NB, i = w % I2::NB;
                    const float2 v = lds[(i + j * I2::NB) * B + bb];
                    return j ? cmulc(v, a.tw_i2[i * (R0 - 1) + j - 1]) : v;
                },
                [&](int w, int k, float2 v) {
                    const int bb = w / I2::NB, i = w % I2::NB, r = tile * B + bb;
                    if (r >= a.keep0 && r < a.keep1) {
                        const gptr<float> dst = as_global(Sm) + static_cast<int64_t>(r - a.keep0) * a.nx;
                        const int c0 = 2 * (i + k * I2::NB);
                        if (EVEN_NX) {
                            if (c0 < a.nx) gstore2_nt(dst + c0, v);
                        } else {
                            if (c0 < a.nx) dst[c0] = v.x;
                            if (c0 + 1 < a.nx) dst[c0 + 1] = v.y;
                        }
                    }
                });
            return;
        }
        float2 y2[I2::S][R0];
        I2::load(y2, lds, tt, b);
        I2::template twiddle<true>(y2, a.tw_i2, tt);
        I2::template butterfly<true>(y2, tt);
        if (rv) {
            const gptr<float> dst = as_global(Sm) + static_cast<int64_t>(row - a.keep0) * a.nx;
#pragma unroll
            for (int s = 0; s < I2::S; ++s) {
                const int i = tt + s * TF;
                if (I2::valid(i)) {
#pragma unroll
                    for (int j = 0; j < R0; ++j) {
                        const int c0 = 2 * (i + j * I2::NB);
                        if (EVEN_NX) {
                            // the map is written once: a streaming store
                            if (c0 < a.nx) gstore2_nt(dst + c0, y2[s][j]);
                        } else {
                            if (c0 < a.nx) dst[c0] = y2[s][j].x;
                            if (c0 + 1 < a.nx) dst[c0 + 1] = y2[s][j].y;
                        }
                    }
                }
            }
        }
    };

    // one tile per workgroup: only tiles with a kept row are dealt out
    const int t0 = (TPW == 1) ? kept_tile(blockIdx.x, ntiles, B, a.keep0, a.keep1) : xcd_tile(blockIdx.x, G);
    if (t0 < 0 || t0 >= ntiles) return;
    const int tt0 = tid0 / B, b0 = tid0 % B;
    if constexpr (TPW == 1) {
        // a tile with no row to keep does nothing (uniform over the workgroup)
        if (t0 * B >= a.keep1 || (t0 + 1) * B <= a.keep0) return;
        float2 xa[R2], xb[R2], xm;
        if constexpr (STG) {
            stage_in(t0);
            __syncthreads();
            load_tile(xa, xb, xm, t0, tt0, b0);
            __syncthreads();  // the first pass rewrites the exchange buffer
        } else {
            load_tile(xa, xb, xm, t0, tt0, b0);
        }
        transform(xa, xb, xm, t0, tt0, b0);
    } else if constexpr (TPW == 2) {
        const int t1 = t0 + G;
        float2 xa[R2], xb[R2], xm, na[R2], nb2[R2], nm;
        load_tile(xa, xb, xm, t0, tt0, b0);
        if (t1 < ntiles) load_tile(na, nb2, nm, t1, tt0, b0);
        transform(xa, xb, xm, t0, tt0, b0);
        if (t1 < ntiles) {
            __syncthreads();
            transform(na, nb2, nm, t1, tt0, b0);
        }
    } else {
        float2 na[R2], nb2[R2], nm;
        load_tile(na, nb2, nm, t0, tt0, b0);
        for (int t = t0; t < ntiles; t += G) {
            const int tid = opaque_v(tid0), tt = tid / B, b = tid % B;
            float2 xa[R2], xb[R2], xm = nm;
#pragma unroll
            for (int j = 0; j < R2; ++j) {
                xa[j] = na[j];
                xb[j] = nb2[j];
            }
            if (t + G < ntiles) load_tile(na, nb2, nm, t + G, tt, b);
            transform(xa, xb, xm, t, tt, b);
            __syncthreads();
        }
    }
}

int row_spec_index(int m, int k)
{
    for (int i = 0; i < kNumRowSpecs; ++i)
        if (kRowSpecs[i].m == m && k-- == 0) return i;
    return -1;
}

int row_spec_count(int m)
{
    int c = 0;
    for (int i = 0; i < kNumRowSpecs; ++i) c += kRowSpecs[i].m == m;
    return c;
}

int row_spec_rows(int idx) { return kRowSpecs[idx].b; }

// Row kernels with the exchanges in two halves (one tile per workgroup): the
// same transforms and layouts as k_rows_r2c_reg / k_rows_c2r_reg, but each
// exchange between passes goes through a float buffer of the same word
// layout twice, real parts then imaginary parts, so the buffer is half the
// size and more workgroups fit on a CU while others wait on HBM.  The
// register allocator plans for exactly OCC waves per SIMD.
template <int M, int TF, int R0, int R1, int R2, int B, int OCC, bool EVEN_NX>
__global__ void __launch_bounds__(TF * B) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_rows_r2c_half(const float *__restrict__ Rm, float2 *__restrict__ W, RowRegArgs a,
                const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    float *f = reinterpret_cast<float *>(lds);
    using F0 = RegPass<M, R0, 1, TF, B, 0>;
    using F1 = RegPass<M, R1, R0, TF, B, R0>;
    constexpr int NB = M / R2;
    static_assert(R0 * R1 * R2 == M && NB / 2 + 1 <= TF, "row specialisation");
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        Rm = it.in;
        W = it.w;
        a.ny = it.ny;
        a.nx = it.nx;
    }
    const int ntiles = (a.ny + B - 1) / B;
    // the item's own tiles are dealt out (in a batch the grid spans the largest item)
    const int t0 = kept_tile(blockIdx.x, ntiles, B, 0, a.ny);
    if (t0 < 0) return;
    const int tt = threadIdx.x / B, b = threadIdx.x % B;
    const int row = t0 * B + b;
    const bool rv = row < a.ny;
    const int64_t ny = a.ny;

    float2 x0[F0::S][R0];
    {
        const gptr<const float> src = as_global(Rm) + static_cast<int64_t>(rv ? row : 0) * a.nx;
#pragma unroll
        for (int s = 0; s < F0::S; ++s) {
            const int i = tt + s * TF;
            if (F0::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) x0[s][j] = load_pair<EVEN_NX>(src, i + j * F0::NB, a.nx, rv);
            }
        }
    }
    F0::template butterfly<false>(x0, tt);
    F0::template store_part<0>(x0, f, tt, b);
    __syncthreads();
    float2 x1[F1::S][R1];
    F1::template load_part<0>(x1, f, tt, b);
    __syncthreads();
    F0::template store_part<1>(x0, f, tt, b);
    __syncthreads();
    F1::template load_part<1>(x1, f, tt, b);
    F1::template twiddle<false>(x1, a.tw_f1, tt);
    F1::template butterfly<false>(x1, tt);
    __syncthreads();
    F1::template store_part<0>(x1, f, tt, b);
    __syncthreads();
    // last pass: thread tt takes butterflies tt and NB - tt (as in k_rows_r2c_reg)
    const bool pairer = tt <= NB / 2;
    const int i1 = tt, i2 = NB - tt;
    const bool two = pairer && (i2 != i1) && (i2 < NB);
    float2 z1[R2], z2[R2];
    if (pairer) {
#pragma unroll
        for (int j = 0; j < R2; ++j) z1[j].x = f[(i1 + j * NB) * B + b];
        if (two) {
#pragma unroll
            for (int j = 0; j < R2; ++j) z2[j].x = f[(i2 + j * NB) * B + b];
        }
    }
    __syncthreads();
    F1::template store_part<1>(x1, f, tt, b);
    __syncthreads();
    if (pairer) {
#pragma unroll
        for (int j = 0; j < R2; ++j) z1[j].y = f[(i1 + j * NB) * B + b];
        if (i1 > 0) {
#pragma unroll
            for (int j = 1; j < R2; ++j) z1[j] = cmul(z1[j], a.tw_f2[i1 * (R2 - 1) + j - 1]);
        }
        dftc<R2, false>(z1);
        if (two) {
#pragma unroll
            for (int j = 0; j < R2; ++j) z2[j].y = f[(i2 + j * NB) * B + b];
#pragma unroll
            for (int j = 1; j < R2; ++j) z2[j] = cmul(z2[j], a.tw_f2[i2 * (R2 - 1) + j - 1]);
            dftc<R2, false>(z2);
        }
        if (rv) {
            // X[k] of this row at ((k / C) * ny + row) * C + k % C
            const int lc = a.lc, cm = (1 << lc) - 1;
            const gptr<float2> dst = as_global(W) + (static_cast<int64_t>(row) << lc);
            auto at = [&](int k) { return ((static_cast<int64_t>(k >> lc) * ny) << lc) + (k & cm); };
            if (i1 == 0) {
#pragma unroll
                for (int j = 0; j < R2; ++j) {
                    const int k = j * NB;
                    gstore2(dst + at(k), r2c_split(z1[j], z1[(R2 - j) % R2], a.rtw[k]));
                }
                gstore2(dst + at(M), r2c_split(z1[0], z1[0], a.rtw[M]));
            } else if (!two) {
#pragma unroll
                for (int j = 0; j < R2; ++j) {
                    const int k = i1 + j * NB;
                    gstore2(dst + at(k), r2c_split(z1[j], z1[R2 - 1 - j], a.rtw[k]));
                }
            } else {
#pragma unroll
                for (int j = 0; j < R2; ++j) {
                    const int k1 = i1 + j * NB, k2 = i2 + j * NB;
                    gstore2(dst + at(k1), r2c_split(z1[j], z2[R2 - 1 - j], a.rtw[k1]));
                    gstore2(dst + at(k2), r2c_split(z2[j], z1[R2 - 1 - j], a.rtw[k2]));
                }
            }
        }
    }
}

template <int M, int TF, int R0, int R1, int R2, int B, int OCC, bool EVEN_NX>
__global__ void __launch_bounds__(TF * B) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_rows_c2r_half(const float2 *__restrict__ W, float *__restrict__ Sm, RowRegArgs a,
                const BatchItem *__restrict__ items)
{
    extern __shared__ float2 lds[];
    float *f = reinterpret_cast<float *>(lds);
    using I1 = RegPass<M, R1, R2, TF, B, R2>;
    using I2 = RegPass<M, R0, R2 * R1, TF, B, 0>;
    constexpr int NB = M / R2;
    static_assert(R0 * R1 * R2 == M && NB / 2 + 1 <= TF, "row specialisation");
    if (items) {
        const BatchItem &it = items[blockIdx.y];
        W = it.w;
        Sm = it.out;
        a.ny = it.ny;
        a.nx = it.nx;
        a.keep0 = it.keep0;
        a.keep1 = it.keep1;
    }
    const int ntiles = (a.ny + B - 1) / B;
    // only tiles with a kept row are dealt out
    const int t0 = kept_tile(blockIdx.x, ntiles, B, a.keep0, a.keep1);
    if (t0 < 0) return;
    // a tile with no row to keep does nothing (uniform over the workgroup)
    if (t0 * B >= a.keep1 || (t0 + 1) * B <= a.keep0) return;
    const int tt = threadIdx.x / B, b = threadIdx.x % B;
    const int row = t0 * B + b;
    const bool rv = row >= a.keep0 && row < a.keep1;
    const int64_t ny = a.ny;
    const bool pairer = tt <= NB / 2;
    const int i1 = tt, i2 = NB - tt;
    const bool two = pairer && (i2 != i1) && (i2 < NB);

    // first pass: thread tt takes butterflies tt and NB - tt, merging X[k]
    // and X[M - k] in registers (as in k_rows_c2r_reg)
    float2 za[R2], zb[R2];
    if (pairer) {
        float2 xa[R2], xb[R2], xm = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < R2; ++j) {
            xa[j] = make_float2(0.f, 0.f);
            xb[j] = make_float2(0.f, 0.f);
        }
        if (rv) {
            const int lc = a.lc, cm = (1 << lc) - 1;
            const gptr<const float2> src = as_global(W) + (static_cast<int64_t>(row) << lc);
            auto at = [&](int k) { return ((static_cast<int64_t>(k >> lc) * ny) << lc) + (k & cm); };
#pragma unroll
            for (int j = 0; j < R2; ++j) xa[j] = gload2(src + at(i1 + j * NB));
            if (two) {
#pragma unroll
                for (int j = 0; j < R2; ++j) xb[j] = gload2(src + at(i2 + j * NB));
            }
            if (i1 == 0) xm = gload2(src + at(M));
        }
        if (i1 == 0) {
#pragma unroll
            for (int j = 0; j < R2; ++j) za[j] = c2r_merge(xa[j], j ? xa[(R2 - j) % R2] : xm, a.rtw[j * NB]);
        } else if (!two) {
#pragma unroll
            for (int j = 0; j < R2; ++j) za[j] = c2r_merge(xa[j], xa[R2 - 1 - j], a.rtw[i1 + j * NB]);
        } else {
#pragma unroll
            for (int j = 0; j < R2; ++j) {
                za[j] = c2r_merge(xa[j], xb[R2 - 1 - j], a.rtw[i1 + j * NB]);
                zb[j] = c2r_merge(xb[j], xa[R2 - 1 - j], a.rtw[i2 + j * NB]);
            }
        }
        dftc<R2, true>(za);
#pragma unroll
        for (int j = 0; j < R2; ++j) f[(i1 * lds_pitch(R2) + j) * B + b] = za[j].x;
        if (two) {
            dftc<R2, true>(zb);
#pragma unroll
            for (int j = 0; j < R2; ++j) f[(i2 * lds_pitch(R2) + j) * B + b] = zb[j].x;
        }
    }
    __syncthreads();
    float2 y1[I1::S][R1];
    I1::template load_part<0>(y1, f, tt, b);
    __syncthreads();
    if (pairer) {
#pragma unroll
        for (int j = 0; j < R2; ++j) f[(i1 * lds_pitch(R2) + j) * B + b] = za[j].y;
        if (two) {
#pragma unroll
            for (int j = 0; j < R2; ++j) f[(i2 * lds_pitch(R2) + j) * B + b] = zb[j].y;
        }
    }
    __syncthreads();
    I1::template load_part<1>(y1, f, tt, b);
    I1::template twiddle<true>(y1, a.tw_i1, tt);
    I1::template butterfly<true>(y1, tt);
    __syncthreads();
    I1::template store_part<0>(y1, f, tt, b);
    __syncthreads();
    float2 y2[I2::S][R0];
    I2::template load_part<0>(y2, f, tt, b);
    __syncthreads();
    I1::template store_part<1>(y1, f, tt, b);
    __syncthreads();
    I2::template load_part<1>(y2, f, tt, b);
    I2::template twiddle<true>(y2, a.tw_i2, tt);
    I2::template butterfly<true>(y2, tt);
    if (rv) {
        const gptr<float> dst = as_global(Sm) + static_cast<int64_t>(row - a.keep0) * a.nx;
#pragma unroll
        for (int s = 0; s < I2::S; ++s) {
            const int i = tt + s * TF;
            if (I2::valid(i)) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int c0 = 2 * (i + j * I2::NB);
                    if (EVEN_NX) {
                        if (c0 < a.nx) gstore2(dst + c0, y2[s][j]);
                    } else {
                        if (c0 < a.nx) dst[c0] = y2[s][j].x;
                        if (c0 + 1 < a.nx) dst[c0 + 1] = y2[s][j].y;
                    }
                }
            }
        }
    }
}

template <int I>
static constexpr size_t row_lds_bytes()
{
    constexpr RowSpec c = kRowSpecs[I];
    // staged: the M + 1 spectrum columns of the tile plus the interleave's pad
    constexpr int w = xchg_words(c.m, c.r0, c.r2);
    constexpr int words = (c.stage && c.m + 2 > w) ? c.m + 2 : w;
    return static_cast<size_t>(words) * c.b * (c.half ? 4 : 8);
}

// SPLIT: the split form of a variant with a matrix-core pass (1 or 2; 0 for
// the other variants)
template <int I, bool FWD, bool EVEN, int SPLIT = (kRowSpecs[I].mf ? 2 : 0)>
static const void *row_fn()
{
    constexpr RowSpec c = kRowSpecs[I];
    static_assert(!c.half || c.pf == 1, "half-exchange rows take one tile per workgroup");
    static_assert(!c.mf || (!c.half && c.pf == 1), "matrix-core rows: full exchange, one tile");
    static_assert((SPLIT != 0) == (c.mf != 0), "split form of a matrix-core variant");
    if constexpr (c.half && FWD)
        return reinterpret_cast<const void *>(&k_rows_r2c_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, EVEN>);
    else if constexpr (c.half)
        return reinterpret_cast<const void *>(&k_rows_c2r_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, EVEN>);
    else if constexpr (FWD)
        return reinterpret_cast<const void *>(
            &k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, c.pf, EVEN, c.stage != 0, SPLIT>);
    else
        return reinterpret_cast<const void *>(
            &k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, c.pf, EVEN, c.stage != 0, SPLIT>);
}

template <int I>
static hipError_t row_attrs_from()
{
    if constexpr (I >= kNumRowSpecs) {
        return hipSuccess;
    } else {
        constexpr int NS = kRowSpecs[I].mf ? 2 : 1;  // instances per direction and parity
        const void *fns[4 * NS];
        if constexpr (kRowSpecs[I].mf) {
            const void *t[8] = {row_fn<I, true, true, 1>(), row_fn<I, true, false, 1>(), row_fn<I, false, true, 1>(),
                                row_fn<I, false, false, 1>(), row_fn<I, true, true, 2>(), row_fn<I, true, false, 2>(),
                                row_fn<I, false, true, 2>(), row_fn<I, false, false, 2>()};
            std::copy(t, t + 8, fns);
        } else {
            const void *t[4] = {row_fn<I, true, true>(), row_fn<I, true, false>(), row_fn<I, false, true>(),
                                row_fn<I, false, false>()};
            std::copy(t, t + 4, fns);
        }
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
            if (e != hipSuccess) return e;
        }
        return row_attrs_from<I + 1>();
    }
}

static hipError_t row_attrs()
{
    static bool attr = false;
    if (attr) return hipSuccess;
    hipError_t e = row_attrs_from<0>();
    if (e == hipSuccess) attr = true;
    return e;
}

template <int I>
static hipError_t launch_row_from(int idx, const void *in, void *out, const RowRegArgs &a0, bool fwd,
                                  hipStream_t s, const BatchItem *items, int nitems)
{
    if constexpr (I >= kNumRowSpecs) {
        return hipErrorInvalidValue;
    } else {
        if (idx != I) return launch_row_from<I + 1>(idx, in, out, a0, fwd, s, items, nitems);
        constexpr RowSpec c = kRowSpecs[I];
        constexpr int PF = c.pf;
        const int ntiles = (a0.ny + c.b - 1) / c.b;
        int groups = PF ? (ntiles + PF - 1) / PF : ntiles;
        if (PF == 0) {
            static int resident[kNumRowSpecs][2] = {};
            int &r = resident[I][fwd ? 0 : 1];
            if (r == 0) {
                int dev = 0, cus = 0, occ = 0;
                const void *f = fwd ? row_fn<I, true, true>() : row_fn<I, false, true>();
                if (hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, c.tf * c.b, row_lds_bytes<I>()) != hipSuccess)
                    return hipErrorInvalidValue;
                r = cus * (occ > 0 ? occ : 1);
            }
            groups = ntiles < r ? ntiles : r;
        }
        // the staged chunks are pairs of columns of the two-column interleave
        if (c.stage && a0.lc != 1) return hipErrorInvalidValue;
        const dim3 g(groups, nitems), t(c.tf * c.b);
        const size_t lds = row_lds_bytes<I>();
        const RowRegArgs &a = a0;
        const bool even = (a.nx % 2) == 0;
        if constexpr (c.half) {
            if (fwd) {
                const float *R = static_cast<const float *>(in);
                float2 *W = static_cast<float2 *>(out);
                if (even) hipLaunchKernelGGL((k_rows_r2c_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, true>), g, t, lds, s, R, W, a, items);
                else hipLaunchKernelGGL((k_rows_r2c_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, false>), g, t, lds, s, R, W, a, items);
            } else {
                const float2 *W = static_cast<const float2 *>(in);
                float *S = static_cast<float *>(out);
                if (even) hipLaunchKernelGGL((k_rows_c2r_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, true>), g, t, lds, s, W, S, a, items);
                else hipLaunchKernelGGL((k_rows_c2r_half<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, false>), g, t, lds, s, W, S, a, items);
            }
        } else if constexpr (c.mf) {
            // the split form picks the instance
            if (!a.mf || (a.split != 1 && a.split != 2)) return hipErrorInvalidValue;
            if (fwd) {
                const float *R = static_cast<const float *>(in);
                float2 *W = static_cast<float2 *>(out);
                if (a.split == 1) {
                    if (even) hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, true, c.stage != 0, 1>), g, t, lds, s, R, W, a, items);
                    else hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, false, c.stage != 0, 1>), g, t, lds, s, R, W, a, items);
                } else {
                    if (even) hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, true, c.stage != 0, 2>), g, t, lds, s, R, W, a, items);
                    else hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, false, c.stage != 0, 2>), g, t, lds, s, R, W, a, items);
                }
            } else {
                const float2 *W = static_cast<const float2 *>(in);
                float *S = static_cast<float *>(out);
                if (a.split == 1) {
                    if (even) hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, true, c.stage != 0, 1>), g, t, lds, s, W, S, a, items);
                    else hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, false, c.stage != 0, 1>), g, t, lds, s, W, S, a, items);
                } else {
                    if (even) hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, true, c.stage != 0, 2>), g, t, lds, s, W, S, a, items);
                    else hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, 1, false, c.stage != 0, 2>), g, t, lds, s, W, S, a, items);
                }
            }
        } else if (fwd) {
            const float *R = static_cast<const float *>(in);
            float2 *W = static_cast<float2 *>(out);
            constexpr bool ST = c.stage != 0;
            if (even) hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, PF, true, ST>), g, t, lds, s, R, W, a, items);
            else hipLaunchKernelGGL((k_rows_r2c_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, PF, false, ST>), g, t, lds, s, R, W, a, items);
        } else {
            const float2 *W = static_cast<const float2 *>(in);
            float *S = static_cast<float *>(out);
            constexpr bool ST = c.stage != 0;
            if (even) hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, PF, true, ST>), g, t, lds, s, W, S, a, items);
            else hipLaunchKernelGGL((k_rows_c2r_reg<c.m, c.tf, c.r0, c.r1, c.r2, c.b, c.occ, PF, false, ST>), g, t, lds, s, W, S, a, items);
        }
        return hipGetLastError();
    }
}

hipError_t launch_rows_r2c_reg(const float *R, float2 *W, const RowRegArgs &a, int idx, hipStream_t s,
                               const BatchItem *items, int nitems)
{
    hipError_t e = set_spec_attributes();
    if (e != hipSuccess) return e;
    return launch_row_from<0>(idx, R, W, a, true, s, items, nitems);
}

hipError_t launch_rows_c2r_reg(const float2 *W, float *S, const RowRegArgs &a, int idx, hipStream_t s,
                               const BatchItem *items, int nitems)
{
    hipError_t e = set_spec_attributes();
    if (e != hipSuccess) return e;
    return launch_row_from<0>(idx, W, S, a, false, s, items, nitems);
}

// Dynamic-LDS limits of every specialised kernel, set once (before any graph
// capture: this is not a stream operation).
hipError_t set_spec_attributes()
{
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = col_attrs_from<0>();
    if (e == hipSuccess) e = row_attrs();
    if (e == hipSuccess) done = true;
    return e;
}

}  // namespace lp
