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
// Blocked intermediate layout: column v of row i sits at
//   W[((v >> logc) * ny + i) << logc | (v & (C-1))],
// so one column block (C adjacent columns, all ny rows) is one contiguous
// run: the column stage reads and writes it with unit stride, and the row
// stages touch C*B*8-byte runs (B rows per workgroup).
//
// Real transforms use the half-length trick: z[n] = x[2n] + i x[2n+1] is
// transformed at length M = Px/2 and split with exp(-2 pi i k/Px).
#include "fft_lds.h"

namespace lp {

// ------------------------------------------------------------------- rows fwd
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
        for (int n = tid; n < m; n += nt) {
            float x0 = 0.f, x1 = 0.f;
            if (row < a.ny) {
                const int c0 = 2 * n;
                if (c0 < a.nx) x0 = src[c0];
                if (c0 + 1 < a.nx) x1 = src[c0 + 1];
            }
            lds[(n << a.logb) + b] = make_float2(x0, x1);
        }
    }
    __syncthreads();
    lds_fft<false>(lds, a.fx, a.logb, a.tw, tid, nt);

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
// FORM 1: real even spectrum, one quadrant stored, (py/2+1) rows per block.
// FORM 2: complex spectrum, py rows per block.  CONJ: use conj(Khat) (the
// transposed operator).
template <int FORM, bool CONJ>
__global__ void __launch_bounds__(1024) k_cols_conv(float2 *__restrict__ W, ColArgs a)
{
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int vb = xcd_tile(blockIdx.x, gridDim.x);
    const int C = 1 << a.logc;
    const int py = a.py;
    const int total = py << a.logc;
    const int stored = a.ny << a.logc;
    float2 *blk = W + static_cast<int64_t>(vb) * stored;

    for (int e = tid; e < total; e += nt)
        lds[e] = (e < stored) ? blk[e] : make_float2(0.f, 0.f);
    __syncthreads();
    lds_fft<false>(lds, a.fy, a.logc, a.tw, tid, nt);

    if constexpr (FORM == 1) {
        const float *kq = static_cast<const float *>(a.kh) + static_cast<int64_t>(vb) * (a.ku << a.logc);
        for (int e = tid; e < total; e += nt) {
            const int u = e >> a.logc, c = e & (C - 1);
            const int uq = (2 * u <= py) ? u : py - u;
            lds[e] = cscale(lds[e], kq[(uq << a.logc) + c]);
        }
    } else {
        const float2 *kc = static_cast<const float2 *>(a.kh) + static_cast<int64_t>(vb) * total;
        for (int e = tid; e < total; e += nt)
            lds[e] = CONJ ? cmulc(lds[e], kc[e]) : cmul(lds[e], kc[e]);
    }
    __syncthreads();
    lds_fft<true>(lds, a.fy, a.logc, a.tw, tid, nt);

    for (int e = tid; e < stored; e += nt) blk[e] = lds[e];
}

// ------------------------------------------------------------------- rows inv
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
    for (int e = tid; e < total; e += nt) {
        const int c = e & (C - 1);
        const int b = (e >> a.logc) & (B - 1);
        const int kb = e >> (a.logc + a.logb);
        const int k = (kb << a.logc) + c;
        const int row = row0 + b;
        if (k < a.h) {
            float2 X = make_float2(0.f, 0.f);
            if (row < a.ny) X = W[((static_cast<int64_t>(kb) * a.ny + row) << a.logc) + c];
            lds[(k << a.logb) + b] = X;
        }
    }
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
    lds_fft<true>(lds, a.fx, a.logb, a.tw, tid, nt);

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
                                                   int form, void *__restrict__ kh)
{
    const int u = blockIdx.y;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ku || v >= (nblk << logc)) return;
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
    const int64_t idx = ((static_cast<int64_t>(vb) * ku + u) << logc) + c;
    if (form == 1)
        static_cast<float *>(kh)[idx] = static_cast<float>(re * scale);
    else
        static_cast<float2 *>(kh)[idx] =
            make_float2(static_cast<float>(re * scale), static_cast<float>(im * scale));
}

// ------------------------------------------------------------------ launchers
static size_t row_lds_bytes(const RowArgs &a) { return static_cast<size_t>(a.m + 1) << a.logb << 3; }

hipError_t launch_rows_r2c(const float *R, float2 *W, const RowArgs &a, int threads, hipStream_t s)
{
    const int groups = (a.ny + (1 << a.logb) - 1) >> a.logb;
    hipLaunchKernelGGL(k_rows_r2c, dim3(groups), dim3(threads), row_lds_bytes(a), s, R, W, a);
    return hipGetLastError();
}

hipError_t launch_rows_c2r(const float2 *W, float *S, const RowArgs &a, int threads, hipStream_t s)
{
    const int groups = (a.ny + (1 << a.logb) - 1) >> a.logb;
    hipLaunchKernelGGL(k_rows_c2r, dim3(groups), dim3(threads), row_lds_bytes(a), s, W, S, a);
    return hipGetLastError();
}

hipError_t launch_cols_conv(float2 *W, const ColArgs &a, int form, bool conj_k, int threads,
                            hipStream_t s)
{
    const size_t lds = static_cast<size_t>(a.py) << a.logc << 3;
    const dim3 g(a.nblk), t(threads);
    if (form == 1)
        hipLaunchKernelGGL((k_cols_conv<1, false>), g, t, lds, s, W, a);
    else if (conj_k)
        hipLaunchKernelGGL((k_cols_conv<2, true>), g, t, lds, s, W, a);
    else
        hipLaunchKernelGGL((k_cols_conv<2, false>), g, t, lds, s, W, a);
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
                            hipStream_t s)
{
    const int ncol = nblk << logc;
    const dim3 g((ncol + 255) / 256, ku), t(256);
    hipLaunchKernelGGL(k_spec_cols, g, t, 0, s, t1, ky, cy, py, ku, h, logc, nblk, taby, scale,
                       form, kh);
    return hipGetLastError();
}

hipError_t set_kernel_attributes()
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_rows_r2c),
        reinterpret_cast<const void *>(&k_rows_c2r),
        reinterpret_cast<const void *>(&k_cols_conv<1, false>),
        reinterpret_cast<const void *>(&k_cols_conv<2, false>),
        reinterpret_cast<const void *>(&k_cols_conv<2, true>),
    };
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lp

// ===================================================== register-resident columns
#include "fft_reg.h"

namespace lp {

// One column per workgroup: forward transform (radices R0, R1, R2), spectrum
// multiply in registers, inverse transform (radices R2, R1, R0; its first
// pass consumes the forward's last-pass outputs straight from registers), and
// only rows < ny read or written.  Column-major intermediate: column v is the
// contiguous run W[v * ny .. v * ny + ny).
template <int N, int TF, int R0, int R1, int R2, int FORM, bool CONJ>
__global__ void __launch_bounds__(((TF + 63) / 64) * 64) k_cols_reg(float2 *__restrict__ W, ColRegArgs a)
{
    extern __shared__ float2 lds[];
    using F0 = RegPass<N, R0, 1, TF, 1>;
    using F1 = RegPass<N, R1, R0, TF, 1>;
    using F2 = RegPass<N, R2, R0 * R1, TF, 1>;
    using I0 = RegPass<N, R2, 1, TF, 1>;
    using I1 = RegPass<N, R1, R2, TF, 1>;
    using I2 = RegPass<N, R0, R2 * R1, TF, 1>;
    const int tt = threadIdx.x;
    const bool act = tt < TF;
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    const int ny = a.ny;
    float2 *col = W + static_cast<int64_t>(v) * ny;

    float2 x0[F0::S][R0];
    if (act) {
#pragma unroll
        for (int s = 0; s < F0::S; ++s) {
            const int i = tt + s * TF;
            if (F0::NB % TF == 0 || i < F0::NB) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int n = i + j * F0::NB;
                    x0[s][j] = (n < ny) ? col[n] : make_float2(0.f, 0.f);
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
        F1::template twiddle<false>(x1, a.tw_f1, tt);
        F1::template butterfly<false>(x1, tt);
    }
    __syncthreads();
    if (act) F1::store(x1, lds, tt, 0);
    __syncthreads();
    float2 x2[F2::S][R2];
    if (act) {
        F2::load(x2, lds, tt, 0);
        F2::template twiddle<false>(x2, a.tw_f2, tt);
        F2::template butterfly<false>(x2, tt);
        // Eq. 9: pixel-wise product with the kernel spectrum, element u = i + j NB
#pragma unroll
        for (int s = 0; s < F2::S; ++s) {
            const int i = tt + s * TF;
            if (F2::NB % TF == 0 || i < F2::NB) {
                if constexpr (FORM == 1) {
                    const float *kq = static_cast<const float *>(a.kh) + static_cast<int64_t>(v) * a.ku;
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const int u = i + j * F2::NB;
                        x2[s][j] = cscale(x2[s][j], kq[(2 * u <= N) ? u : N - u]);
                    }
                } else {
                    const float2 *kc = static_cast<const float2 *>(a.kh) + static_cast<int64_t>(v) * N;
#pragma unroll
                    for (int j = 0; j < R2; ++j) {
                        const float2 k = kc[i + j * F2::NB];
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
        I1::template twiddle<true>(y1, a.tw_i1, tt);
        I1::template butterfly<true>(y1, tt);
    }
    __syncthreads();
    if (act) I1::store(y1, lds, tt, 0);
    __syncthreads();
    if (act) {
        float2 y2[I2::S][R0];
        I2::load(y2, lds, tt, 0);
        I2::template twiddle<true>(y2, a.tw_i2, tt);
        I2::template butterfly<true>(y2, tt);
#pragma unroll
        for (int s = 0; s < I2::S; ++s) {
            const int i = tt + s * TF;
            if (I2::NB % TF == 0 || i < I2::NB) {
#pragma unroll
                for (int j = 0; j < R0; ++j) {
                    const int n = i + j * I2::NB;
                    if (n < ny) col[n] = y2[s][j];
                }
            }
        }
    }
}

int col_spec_index(int n)
{
    for (int i = 0; i < static_cast<int>(sizeof kColSpecs / sizeof kColSpecs[0]); ++i)
        if (kColSpecs[i].n == n) return i;
    return -1;
}

size_t col_spec_lds_bytes(int n) { return static_cast<size_t>(lds_words(n)) * 8; }

template <int I>
static hipError_t launch_col_spec(float2 *W, const ColRegArgs &a, int ncols, int form, bool conj_k,
                                  hipStream_t s)
{
    constexpr ColSpec c = kColSpecs[I];
    const dim3 g(ncols), t(((c.tf + 63) / 64) * 64);
    const size_t lds = col_spec_lds_bytes(c.n);
    if (form == 1)
        hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 1, false>), g, t, lds, s, W, a);
    else if (conj_k)
        hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 2, true>), g, t, lds, s, W, a);
    else
        hipLaunchKernelGGL((k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 2, false>), g, t, lds, s, W, a);
    return hipGetLastError();
}

template <int I>
static hipError_t set_col_spec_attr()
{
    constexpr ColSpec c = kColSpecs[I];
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 1, false>),
        reinterpret_cast<const void *>(&k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 2, false>),
        reinterpret_cast<const void *>(&k_cols_reg<c.n, c.tf, c.r0, c.r1, c.r2, 2, true>),
    };
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_cols_reg(float2 *W, const ColRegArgs &a, int n, int ncols, int form, bool conj_k,
                           hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e;
        if ((e = set_col_spec_attr<0>()) != hipSuccess || (e = set_col_spec_attr<1>()) != hipSuccess ||
            (e = set_col_spec_attr<2>()) != hipSuccess || (e = set_col_spec_attr<3>()) != hipSuccess)
            return e;
        attr = true;
    }
    switch (col_spec_index(n)) {
        case 0: return launch_col_spec<0>(W, a, ncols, form, conj_k, s);
        case 1: return launch_col_spec<1>(W, a, ncols, form, conj_k, s);
        case 2: return launch_col_spec<2>(W, a, ncols, form, conj_k, s);
        case 3: return launch_col_spec<3>(W, a, ncols, form, conj_k, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lp
