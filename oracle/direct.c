/*
 * Plain FP64 direct-sum oracle for the night-sky-brightness convolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * What it computes (Bara et al. 2019, Sec. 2.3, Eq. 7 discretised on the
 * pixel grid, with the zero padding of Sec. 2.5): for a radiance grid R of
 * ny x nx pixels and a point-spread matrix K of ky x kx pixels whose centre
 * sits at (cy, cx) = ((ky-1)/2, (kx-1)/2) (integer division),
 *
 *   S_full(i,j) = sum_{a<ky} sum_{b<kx} K(a,b) R(i-a, j-b),
 *                 0 <= i < ny+ky-1, 0 <= j < nx+kx-1,        R = 0 off-grid
 *   S(i,j)      = S_full(i+cy, j+cx),   0 <= i < ny, 0 <= j < nx  ("same")
 *   A(p,q)      = sum_{i<ny} sum_{j<nx} G(i,j) K(i+cy-p, j+cx-q)
 *                 (the transpose of the "same" operator; K = 0 off-support)
 *
 * The output map has the input's size, as in the paper's results section.
 * No area element is applied: the pitch squared, if wanted, is folded into K.
 * Arithmetic is plain FP64 accumulation in natural loop order; there is no
 * blocking, reordering or transform of any kind.
 *
 * Arrays are row-major.  Every function returns 0 on success and -1 on a
 * bad argument (non-positive size or null pointer).
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int bad_sizes(int64_t ny, int64_t nx, int64_t ky, int64_t kx)
{
    return ny <= 0 || nx <= 0 || ky <= 0 || kx <= 0;
}

/* One output pixel of the full linear convolution (Eq. 7 as a pixel sum). */
static double full_pixel(const double *R, int64_t ny, int64_t nx,
                         const double *K, int64_t ky, int64_t kx,
                         int64_t i, int64_t j)
{
    double s = 0.0;
    for (int64_t a = 0; a < ky; ++a) {
        int64_t r = i - a;
        if (r < 0 || r >= ny)
            continue;
        for (int64_t b = 0; b < kx; ++b) {
            int64_t c = j - b;
            if (c < 0 || c >= nx)
                continue;
            s += K[a * kx + b] * R[r * nx + c];
        }
    }
    return s;
}

/* Full linear convolution, (ny+ky-1) x (nx+kx-1) output. */
int orc_conv_full(const double *R, int64_t ny, int64_t nx,
                  const double *K, int64_t ky, int64_t kx, double *S)
{
    if (!R || !K || !S || bad_sizes(ny, nx, ky, kx))
        return -1;
    int64_t my = ny + ky - 1, mx = nx + kx - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < my; ++i)
        for (int64_t j = 0; j < mx; ++j)
            S[i * mx + j] = full_pixel(R, ny, nx, K, ky, kx, i, j);
    return 0;
}

/* "Same" convolution: the ny x nx window of the full one starting at
 * (cy, cx), i.e. aligned on the kernel centre. */
int orc_conv_same(const double *R, int64_t ny, int64_t nx,
                  const double *K, int64_t ky, int64_t kx, double *S)
{
    if (!R || !K || !S || bad_sizes(ny, nx, ky, kx))
        return -1;
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < nx; ++j)
            S[i * nx + j] = full_pixel(R, ny, nx, K, ky, kx, i + cy, j + cx);
    return 0;
}

/* "Same" convolution at a list of flat pixel indices p = i*nx + j. */
int orc_conv_same_pixels(const double *R, int64_t ny, int64_t nx,
                         const double *K, int64_t ky, int64_t kx,
                         const int64_t *idx, int64_t n, double *out)
{
    if (!R || !K || (n > 0 && (!idx || !out)) || bad_sizes(ny, nx, ky, kx) || n < 0)
        return -1;
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
    for (int64_t t = 0; t < n; ++t)
        if (idx[t] < 0 || idx[t] >= ny * nx)
            return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = idx[t] / nx, j = idx[t] % nx;
        out[t] = full_pixel(R, ny, nx, K, ky, kx, i + cy, j + cx);
    }
    return 0;
}

/* One pixel of the transposed "same" operator. */
static double adjoint_pixel(const double *G, int64_t ny, int64_t nx,
                            const double *K, int64_t ky, int64_t kx,
                            int64_t p, int64_t q)
{
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
    double s = 0.0;
    for (int64_t i = 0; i < ny; ++i) {
        int64_t a = i + cy - p;
        if (a < 0 || a >= ky)
            continue;
        for (int64_t j = 0; j < nx; ++j) {
            int64_t b = j + cx - q;
            if (b < 0 || b >= kx)
                continue;
            s += G[i * nx + j] * K[a * kx + b];
        }
    }
    return s;
}

/* Transpose of the "same" operator applied to an ny x nx map G. */
int orc_adjoint_same(const double *G, int64_t ny, int64_t nx,
                     const double *K, int64_t ky, int64_t kx, double *A)
{
    if (!G || !K || !A || bad_sizes(ny, nx, ky, kx))
        return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < ny; ++p)
        for (int64_t q = 0; q < nx; ++q)
            A[p * nx + q] = adjoint_pixel(G, ny, nx, K, ky, kx, p, q);
    return 0;
}

/* Transposed operator at a list of flat pixel indices. */
int orc_adjoint_same_pixels(const double *G, int64_t ny, int64_t nx,
                            const double *K, int64_t ky, int64_t kx,
                            const int64_t *idx, int64_t n, double *out)
{
    if (!G || !K || (n > 0 && (!idx || !out)) || bad_sizes(ny, nx, ky, kx) || n < 0)
        return -1;
    for (int64_t t = 0; t < n; ++t)
        if (idx[t] < 0 || idx[t] >= ny * nx)
            return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n; ++t)
        out[t] = adjoint_pixel(G, ny, nx, K, ky, kx, idx[t] / nx, idx[t] % nx);
    return 0;
}

/* Transposed operator applied to a map that is zero except at n sites
 * (flat indices `site`, values g): A(p,q) = sum_t g_t K(i_t+cy-p, j_t+cx-q).
 * This is the gradient of a loss that depends on S only at the sites. */
int orc_adjoint_sparse(const int64_t *site, const double *g, int64_t n,
                       int64_t ny, int64_t nx,
                       const double *K, int64_t ky, int64_t kx, double *A)
{
    if (!K || !A || (n > 0 && (!site || !g)) || n < 0 || bad_sizes(ny, nx, ky, kx))
        return -1;
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
    for (int64_t t = 0; t < n; ++t)
        if (site[t] < 0 || site[t] >= ny * nx)
            return -1;
    for (int64_t p = 0; p < ny * nx; ++p)
        A[p] = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = site[t] / nx, j = site[t] % nx;
        for (int64_t a = 0; a < ky; ++a) {
            int64_t p = i + cy - a;
            if (p < 0 || p >= ny)
                continue;
            for (int64_t b = 0; b < kx; ++b) {
                int64_t q = j + cx - b;
                if (q < 0 || q >= nx)
                    continue;
                A[p * nx + q] += g[t] * K[a * kx + b];
            }
        }
    }
    return 0;
}

/* "Same" convolution with a separable kernel K(a,b) = u(a) v(b): a 1-D
 * convolution of every row with v, then of every column with u, each with
 * the centre convention above.  It is the definition above with the double
 * sum factored, and lets a full-field reference be formed at map sizes where
 * the 2-D sum would take hours. */
int orc_conv_same_separable(const double *R, int64_t ny, int64_t nx,
                            const double *u, int64_t ky,
                            const double *v, int64_t kx,
                            double *T, double *S)
{
    if (!R || !u || !v || !T || !S || bad_sizes(ny, nx, ky, kx))
        return -1;
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
    /* rows: T(i,j) = sum_b v(b) R(i, j+cx-b) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < nx; ++j) {
            double s = 0.0;
            for (int64_t b = 0; b < kx; ++b) {
                int64_t c = j + cx - b;
                if (c < 0 || c >= nx)
                    continue;
                s += v[b] * R[i * nx + c];
            }
            T[i * nx + j] = s;
        }
    /* columns: S(i,j) = sum_a u(a) T(i+cy-a, j) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ny; ++i) {
        for (int64_t j = 0; j < nx; ++j)
            S[i * nx + j] = 0.0;
        for (int64_t a = 0; a < ky; ++a) {
            int64_t r = i + cy - a;
            if (r < 0 || r >= ny)
                continue;
            for (int64_t j = 0; j < nx; ++j)
                S[i * nx + j] += u[a] * T[r * nx + j];
        }
    }
    return 0;
}

/* Separable "same" convolution at sampled pixels (row pass done per pixel
 * only over the rows that the column pass touches). */
int orc_conv_same_separable_pixels(const double *R, int64_t ny, int64_t nx,
                                   const double *u, int64_t ky,
                                   const double *v, int64_t kx,
                                   const int64_t *idx, int64_t n, double *out)
{
    if (!R || !u || !v || (n > 0 && (!idx || !out)) || n < 0 || bad_sizes(ny, nx, ky, kx))
        return -1;
    int64_t cy = (ky - 1) / 2, cx = (kx - 1) / 2;
    for (int64_t t = 0; t < n; ++t)
        if (idx[t] < 0 || idx[t] >= ny * nx)
            return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = idx[t] / nx, j = idx[t] % nx;
        double s = 0.0;
        for (int64_t a = 0; a < ky; ++a) {
            int64_t r = i + cy - a;
            if (r < 0 || r >= ny)
                continue;
            double row = 0.0;
            for (int64_t b = 0; b < kx; ++b) {
                int64_t c = j + cx - b;
                if (c < 0 || c >= nx)
                    continue;
                row += v[b] * R[r * nx + c];
            }
            s += u[a] * row;
        }
        out[t] = s;
    }
    return 0;
}

/* Number of threads the OpenMP runtime will use (0 when built without it). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads the OpenMP loops use from now on (n >= 1);
 * returns the number in effect. */
int orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
