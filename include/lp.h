/*
 * lp.h -- C ABI of the MI355X (gfx950) FFT evaluation of artificial
 * night-sky-brightness maps.
 *
 * Method (Bara, Falchi, Furgoni, Lima 2019, "Fast Fourier-transform
 * calculation of artificial night sky brightness maps"):
 *   - for factorable sources (Sec. 2.2, Eq. 3) and a shift-invariant
 *     point-spread function (Sec. 2.3), the sky-brightness map B is the 2-D
 *     convolution of the ground radiance L1 with the kernel K (Eq. 7);
 *   - it is evaluated through the convolution theorem (Eq. 9) with the 2-D
 *     DFT of Eq. 10, after zero padding both matrices to at least
 *     N_L + N_K - 1 rows and columns so the circular convolution equals the
 *     linear one (Sec. 2.5, Fig. 1);
 *   - the output map has the input's size (Sec. 3).
 *
 * Discrete statement computed here, for a radiance grid R (ny x nx) and a
 * kernel K (ky x kx) with centre (cy, cx) = ((ky-1)/2, (kx-1)/2):
 *     S(i,j) = sum_{a<ky, b<kx} K(a,b) R(i+cy-a, j+cx-b),  0<=i<ny, 0<=j<nx,
 * with R = 0 outside the grid.  K(a,b) is the kernel at observer-minus-source
 * displacement ((a-cy) pitch, (b-cx) pitch).  No area element is applied (the
 * caller folds pitch^2 into K if wanted).
 *
 * Conventions for every call:
 *   - arrays are row-major and dense;
 *   - "device" pointers are HIP device memory on the current device, owned by
 *     the caller; "host" pointers are ordinary host memory owned by the
 *     caller;
 *   - calls that take device data enqueue work on the stream given to
 *     lp_plan_bind / lp_batch_bind and return without synchronising; errors
 *     in that work surface at the caller's next synchronisation;
 *   - a plan (or batch) is not safe for concurrent use from several host
 *     threads; use one per stream;
 *   - on failure a call returns a negative lp_status (or NULL) and
 *     lp_last_error() describes it; argument checks happen before any HIP
 *     call, so a rejected call has no device side effects.
 */
#ifndef LP_H
#define LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_plan lp_plan;   /* opaque: one map shape + one kernel */
typedef struct lp_batch lp_batch; /* opaque: many tiles, several kernels */

typedef enum lp_status {
    LP_OK = 0,
    LP_E_INVALID = -1, /* size <= 0, null pointer, bad pitch, non-finite kernel */
    LP_E_SIZE = -2,    /* padding too small, not 5-smooth, or beyond the maximum */
    LP_E_STATE = -3,   /* call out of order (e.g. convolve before spectrum)      */
    LP_E_NOMEM = -4,   /* workspace unbound or too small                         */
    LP_E_DEVICE = -5   /* a HIP runtime or launch error                          */
} lp_status;

/* Spectrum storage forms (lp_plan_spectrum_form). */
enum { LP_FORM_NONE = 0, LP_FORM_REAL_QUADRANT = 1, LP_FORM_COMPLEX = 2 };

/* Largest padded sizes a plan accepts.  Half a padded row plus one must fit
 * one workgroup's LDS (Px/2 + 1 <= 20480 complex FP32 values).  A padded
 * column up to 20480 values is transformed within one workgroup; a longer
 * one (up to LP_MAX_PY) goes through the four-step column stage: Py = P1 P2
 * with P2 <= 20480, three passes over a Py-long scratch column per stored
 * column (lp_plan_column_split reports the split).  Four-step plans take one
 * source class and run their column stage in FP32. */
#define LP_MAX_PY 131072
#define LP_MAX_PX 40958

/* Text description of the last failure on this host thread ("" if none).
 * The pointer stays valid until the next lp_* call on the same thread. */
const char *lp_last_error(void);

/* lp_status of the last failure on this host thread (LP_OK if the last call
 * succeeded); lets a caller classify a NULL from lp_plan_create. */
int lp_last_status(void);

/* Library version string. */
const char *lp_version(void);

/* ---------------------------------------------------------------- plans --
 * lp_plan_create: a plan for maps of ny x nx pixels and kernels of ky x kx
 * pixels on a grid of pitch_km (Eq. 7, Sec. 2.5).  Host only; no HIP call.
 * The padded size defaults, per axis, to the smallest number 2^a 3^b 5^c that
 * is >= n + k - 1 (the common size of Sec. 2.5), and even along x.
 * Returns NULL on error (sizes <= 0, pitch <= 0 or non-finite: LP_E_INVALID;
 * n + floor(k/2) above LP_MAX_PY / LP_MAX_PX: LP_E_SIZE). */
lp_plan *lp_plan_create(int64_t ny, int64_t nx, int64_t ky, int64_t kx, double pitch_km);

/* Free the plan (host memory only; the bound workspace stays the caller's).
 * NULL is accepted. */
void lp_plan_destroy(lp_plan *plan);

/* Override the padded size.  Sec. 2.5 pads to n + k - 1, the extent of the
 * full linear convolution; the input-sized output window (Sec. 3) needs only
 * n + floor(k/2) per axis: with that length a kernel tap that wraps round
 * the circular transform always lands in the zero padding, so the window is
 * unchanged (beyond round-off) for any padding from there up.
 * py >= ny + floor(ky/2) and px >= nx + floor(kx/2), both 5-smooth, px even,
 * py <= LP_MAX_PY, px <= LP_MAX_PX (else LP_E_SIZE).  Must precede
 * lp_plan_bind (else LP_E_STATE).  lp_plan_create's default is the smallest
 * such size >= n + k - 1, or >= n + floor(k/2) where that exceeds the maximum. */
int lp_plan_set_padding(lp_plan *plan, int64_t py, int64_t px);

/* Current padded size into *py, *px (host pointers). */
int lp_plan_get_padding(const lp_plan *plan, int64_t *py, int64_t *px);

/* Device workspace the plan needs, in bytes (0 for a NULL plan): the
 * intermediate spectra of the map (two copies where the padded column
 * length has specialised kernels, which write the column stage's result out
 * of place), the stored kernel spectrum and the FP32 twiddle tables.
 * Depends on the padding. */
size_t lp_plan_workspace_bytes(const lp_plan *plan);

/* Attach caller-owned device memory (dev_ws, >= lp_plan_workspace_bytes,
 * 256-byte aligned) and a stream (a hipStream_t; NULL = the null stream).
 * Uploads the twiddle tables (async on that stream).  May be called again to
 * move the plan to another workspace or stream; the kernel spectrum must then
 * be computed again.  LP_E_NOMEM if bytes is too small. */
int lp_plan_bind(lp_plan *plan, void *dev_ws, size_t bytes, void *stream);

/* Kernel spectrum (Fig. 1 "FFT(K)", Eq. 9, Eq. 10): K is placed wrap-centred
 * in the Py x Px padded grid, transformed by a direct FP64 DFT on the device,
 * scaled by 1/(Py Px), rounded once to FP32 and kept in the workspace.  If K
 * is exactly mirror-symmetric on both axes with odd sizes, its spectrum is
 * real and even and only one real quadrant is stored; otherwise the complex
 * Hermitian half.  psf: host, FP64, ky*kx row-major, read during the call
 * only.  Synchronises the bound stream before returning.  Errors:
 * LP_E_INVALID (null, NaN or Inf entries), LP_E_STATE (not bound). */
int lp_kernel_spectrum(lp_plan *plan, const double *psf);

/* Which spectrum form the plan holds (LP_FORM_*). */
int lp_plan_spectrum_form(const lp_plan *plan);

/* Copy the stored spectrum to host memory in natural order as FP32 complex
 * pairs, out[(u * (Px/2+1) + v) * 2 + {0: re, 1: im}] for 0<=u<Py,
 * 0<=v<=Px/2, already scaled by 1/(Py Px).  Synchronises the bound stream.
 * out must hold Py*(Px/2+1)*2 floats. */
int lp_plan_read_spectrum(lp_plan *plan, float *out);

/* The hot path: S = K (*) R cropped to ny x nx (Eq. 7 via Eq. 9).
 * radiance: device FP32 ny*nx; out: device FP32 ny*nx (may alias radiance).
 * Three kernels on the bound stream: rows forward real-to-complex transform
 * with implicit zero padding; per-column forward transform, multiply by the
 * kernel spectrum, inverse transform; rows inverse complex-to-real transform
 * with the crop.  Non-finite radiance is not checked (one NaN spreads over
 * the whole map through the transform).  Errors: LP_E_INVALID (null),
 * LP_E_STATE (no spectrum), LP_E_NOMEM (unbound), LP_E_DEVICE. */
int lp_convolve(lp_plan *plan, const float *radiance, float *out);

/* For callers that cannot allocate device memory at call time (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * lp_convolve with the intermediate spectra of the map held in a scratch
 * array that is part of the library itself (a device-resident array of
 * LP_NOALLOC_MAX_BYTES on each GPU the library runs on, kept until the
 * process ends) instead of in the bound workspace; the column stage then
 * works in place in that array.  Same arguments, same kernels and
 * arithmetic, same result bits as lp_convolve; the plan must still be bound
 * (its workspace holds the kernel spectrum and the twiddle tables) and its
 * workspace must be on the current device.  The call allocates nothing: no
 * hipMalloc, no allocating library routine.  Every call on one GPU shares
 * that GPU's array, which keeps the last call's contents (nothing in it
 * needs to start at zero): calls that overlap on one GPU -- from several
 * plans, streams or host threads at once -- race and give wrong results;
 * serialise them.  Errors: LP_E_INVALID (null, or the workspace on another
 * device), LP_E_STATE (no spectrum, several classes), LP_E_SIZE (the
 * intermediate, (Px/2+1 rounded up to even) * ny * 8 bytes, exceeds
 * LP_NOALLOC_MAX_BYTES, or the padded columns take the four-step stage,
 * whose scratch lives in the workspace), LP_E_NOMEM (unbound),
 * LP_E_DEVICE. */
#define LP_NOALLOC_MAX_BYTES (128u << 20)
int lp_convolve_noalloc(lp_plan *plan, const float *radiance, float *out);

/* Transpose of lp_convolve, for gradients: grad_in = C^T grad_out, where C
 * is the discrete form of Eq. 7 that lp_convolve evaluates, so
 * grad_in(p, q) = sum_{i,j} grad_out(i, j) K(i + cy - p, j + cx - q), a
 * correlation with K.  By Eq. 9 it is the same three stages with the
 * conjugate of the stored spectrum (the crop and the zero padding swap
 * roles, which the implicit padding covers).  Device FP32 ny*nx in and out
 * (may alias).  Same errors as lp_convolve. */
int lp_adjoint(lp_plan *plan, const float *grad_out, float *grad_in);

/* ------------------------------------------------------ source classes --
 * Sources grouped into T classes, each factorable with its own angular and
 * spectral pattern (Sec. 2.2, Eq. 4): class t has its own radiance map L_1t
 * and its own kernel K_t (Eq. 6 with L_2t), and the sky brightness is
 * B = sum_t K_t (*) L_1t.  The products of Eq. 9 are summed in the Fourier
 * domain, so the T maps share one inverse transform.
 * lp_plan_set_classes: 1 <= T <= LP_MAX_CLASSES, before lp_plan_bind
 * (LP_E_STATE after); the workspace then holds T intermediates and T
 * spectra.  On a plan with T > 1, lp_kernel_spectrum, lp_convolve and
 * lp_adjoint return LP_E_STATE.  lp_plan_classes: T (-1 for NULL). */
#define LP_MAX_CLASSES 16
int lp_plan_set_classes(lp_plan *plan, int n_classes);
int lp_plan_classes(const lp_plan *plan);

/* Spectra of the T kernels (host array of T host pointers, each FP64
 * ky*kx row-major; read during the call only), computed as
 * lp_kernel_spectrum does; one storage form for all: the real quadrant only
 * if every kernel is mirror-symmetric.  Synchronises the bound stream.
 * Errors as lp_kernel_spectrum. */
int lp_kernel_spectra(lp_plan *plan, const double *const *psfs);

/* B = sum_t K_t (*) L_1t cropped to ny x nx.  radiance: host array of T
 * device pointers to FP32 ny*nx maps; out: device FP32 ny*nx (may alias any
 * of them).  The rows forward stage runs once per class, the column stage
 * transforms each class, multiplies by its spectrum and sums before one
 * inverse transform, the rows inverse stage runs once.  Errors as
 * lp_convolve. */
int lp_convolve_classes(lp_plan *plan, const float *const *radiance, float *out);

/* Gradient with respect to class cls's map: grad_in = C_cls^T grad_out
 * (lp_adjoint with kernel cls).  Device FP32 ny*nx in and out (may alias).
 * LP_E_INVALID for cls outside [0, T). */
int lp_adjoint_class(lp_plan *plan, int cls, const float *grad_out, float *grad_in);

/* Debug mode for reads of memory that no stage wrote.
 * With enable != 0, every later call on the plan first fills its
 * intermediate spectra (all classes and the column stage's output copy, or
 * the no-allocation scratch array) and the four-step scratch with a quiet
 * NaN, by a kernel on the bound stream;
 * an element that any stage read before a stage wrote it would turn the
 * output into NaN, so a poisoned run must give the same bits as an ordinary
 * one.  Costs one fill of the intermediate per call.  New plans start with
 * it on when the environment variable LP_DEBUG_POISON is set and not "0".
 * Errors: LP_E_INVALID. */
int lp_plan_set_poison(lp_plan *plan, int enable);

/* Per-stage timing with HIP events on the bound stream.  enable = N > 0
 * starts recording events around each of the three stages of every N-th
 * call that runs the path (lp_convolve, lp_adjoint, lp_convolve_classes,
 * lp_adjoint_class), counting from the next one (up to 1024 recorded calls
 * are kept); 0 stops; N < 0 is
 * LP_E_INVALID.  The four events of a recorded call add some microseconds to
 * it, so a caller timing many calls can sample them with N > 1.
 * lp_plan_stage_ms synchronises on the last event, writes the summed
 * milliseconds of stage s (0: rows forward, 1: columns, 2: rows inverse) of
 * the recorded calls to ms[s] for s < n, their number to *calls, and clears
 * the record. */
int lp_plan_timing(lp_plan *plan, int enable);
int lp_plan_stage_ms(lp_plan *plan, double *ms, int n, int *calls);

/* Kernel family of the three stages.  LP_KERNELS_AUTO (default): for each
 * stage, a register-resident kernel specialised at compile time for the
 * padded column length (column stage) or half row length (row stages) when
 * the library has one -- three large-radix passes, the spectrum multiply and
 * the real-to-complex split in registers -- else the generic LDS-staged
 * kernel; LP_KERNELS_GENERIC: always the generic ones.  lp_plan_kernels
 * reports LP_KERNELS_SPECIALISED if lp_convolve runs at least one specialised
 * stage, else LP_KERNELS_GENERIC (-1 for a NULL plan). */
enum { LP_KERNELS_AUTO = 0, LP_KERNELS_GENERIC = 1, LP_KERNELS_SPECIALISED = 2 };
int lp_plan_set_kernels(lp_plan *plan, int which);
int lp_plan_kernels(const lp_plan *plan);

/* Variants (autotuning).  The library holds several compile-time
 * specialisations for some lengths (different radix orders, threads per
 * transform, transforms per workgroup, persistence with register prefetch);
 * a plan starts on variant 0 of each stage.  lp_plan_variant_count: how many
 * exist for the plan's padded size and precision (0: none, the generic
 * kernel runs).
 * lp_plan_set_variant may be called at any time (after lp_plan_bind it
 * re-uploads the stage's twiddle tables and synchronises the stream).
 * lp_plan_variant_info writes up to n of {R0, R1, R2, threads per transform,
 * transforms per workgroup, min waves per SIMD, tiles per workgroup (0: a
 * persistent loop; always 1 for the column stage), length, half exchange
 * (1: the passes exchange real and imaginary parts through LDS separately,
 * halving the buffer so that twice as many workgroups fit on a CU), staged
 * (row stages: 1 if the intermediate moves between HBM and LDS in 16-byte
 * chunks of two spectrum columns), matrix core (1 if the radix-16 pass R0 runs
 * on the matrix cores in the plan's split form)}.  The variants of a
 * split-precision plan are those with a matrix-core pass, and those of an
 * FP32 plan the others, so the count and numbering depend on
 * lp_plan_set_precision (which resets every stage to variant 0).
 * LP_STAGE_ROWS selects the variant of both row stages (and reports the
 * forward one); LP_STAGE_ROWS_INVERSE the inverse row stage alone, so the
 * two directions may run different specialisations of the same length. */
enum { LP_STAGE_ROWS = 0, LP_STAGE_COLUMNS = 1, LP_STAGE_ROWS_INVERSE = 2 };
int lp_plan_variant_count(const lp_plan *plan, int stage);
int lp_plan_get_variant(const lp_plan *plan, int stage);
int lp_plan_set_variant(lp_plan *plan, int stage, int k);
int lp_plan_variant_info(const lp_plan *plan, int stage, int k, int *info, int n);

/* Launch shape the plan chose (host pointers, any may be NULL): columns per
 * workgroup of the column stage, rows per workgroup of the row stages. */
int lp_plan_shape(const lp_plan *plan, int *cols_per_group, int *rows_per_group);

/* Column transform split of the plan: *p1 = 1, *p2 = Py when a padded column
 * fits one workgroup's LDS; otherwise the four-step factors Py = P1 * P2
 * (P2 the largest divisor of Py up to 20480: Cooley-Tukey's split of one
 * length-Py DFT into P2 DFTs of length P1 and P1 of length P2, twiddled by
 * exp(-2 pi i n2 k1 / Py) between them).  Host pointers; LP_E_INVALID on
 * NULL. */
int lp_plan_column_split(const lp_plan *plan, int64_t *p1, int64_t *p2);

/* Arithmetic of the transforms (the DFTs of Eq. 10 inside Eq. 9).
 * LP_PRECISION_FP32 (default): every butterfly on the vector ALU in FP32.
 * The split forms run radix-16 passes as dense 32 x 32 real matrix products
 * on the matrix cores (v_mfma_f32_16x16x32, FP32 accumulation), with both
 * operands split into low-precision terms:
 *   LP_PRECISION_SPLIT_FP16: x = hi + lo in FP16 after scaling each
 *     butterfly's 16 inputs by a power of two (largest in [2^14, 2^15)), the
 *     matrix by 2^14; three products hi*hi + hi*lo + lo*hi;
 *   LP_PRECISION_SPLIT_BF16: x = x1 + x2 + x3 in BF16, six products (all
 *     terms of total order <= 4).
 * Both keep the dropped terms near 2^-22 of a butterfly's largest input, so
 * the result stays at FP32-level error.  A split plan runs each stage on a
 * register-resident specialisation whose radix-16 pass is on the matrix
 * cores where the library has one for the length (9216-point half rows and
 * 18432-point columns: the radix-16 pass is the forward transform's first
 * and the inverse's last), else on the generic LDS-staged kernels, which
 * take every radix-16 pass of the length to the matrix cores (four-step
 * columns keep FP32 middle transforms).  Lengths without a factor 16 get no
 * matrix pass.  Set before lp_plan_bind (LP_E_STATE after);
 * unknown mode: LP_E_INVALID.  lp_plan_precision returns the mode (-1 for a
 * NULL plan). */
enum { LP_PRECISION_FP32 = 0, LP_PRECISION_SPLIT_FP16 = 1, LP_PRECISION_SPLIT_BF16 = 2 };
int lp_plan_set_precision(lp_plan *plan, int mode);
int lp_plan_precision(const lp_plan *plan);

/* ------------------------------------------------------- reprojection --
 * Sec. 2.4: the radiance composites come on a uniform longitude-latitude
 * grid whose ground scale varies with latitude; the convolution needs a grid
 * of uniform scale (shift-invariant kernel), so the map is reprojected onto a
 * transverse Mercator (UTM-type) grid by nearest-neighbour resampling.
 *
 * Source grid: row r has latitude lat_first - r * dlat, column c longitude
 * lon_first + c * dlon (degrees, pixel centres; rows run southward).
 * Projected grid: row i has northing y_first - i * pitch, column j easting
 * x_first + j * pitch (km from the equator and from the central meridian
 * lon0; no false easting or northing), central scale k0, sphere radius R.
 * Each projected pixel centre is mapped to latitude and longitude by the
 * spherical inverse transverse Mercator (Snyder; the paper's reference for
 * Eq. 11) and takes the nearest source pixel in (row, column) index space,
 * halves rounded to even; 0 where that pixel lies outside the source grid.
 * ground_area != 0 multiplies by 1 / k^2, k = k0 cosh(x / (k0 R)) (Eq. 11):
 * the projection is conformal, so a projected cell of pitch^2 covers
 * pitch^2 / k^2 of ground (a radiance map becomes flux per cell / pitch^2).
 * FP64 index arithmetic.  src and dst: device FP32, row-major, not
 * overlapping; the call enqueues one kernel on `stream` (a hipStream_t;
 * NULL = the null stream) and returns.  Errors: LP_E_INVALID (null pointers,
 * sizes <= 0, non-finite or non-positive steps, pitch, k0 or R), LP_E_SIZE
 * (more than 262140 projected rows), LP_E_DEVICE. */
typedef struct {
    int64_t rows, cols;
    double lat_first_deg, lon_first_deg, dlat_deg, dlon_deg;
} lp_latlon_grid;
typedef struct {
    int64_t rows, cols;
    double x_first_km, y_first_km, pitch_km;
    double lon0_deg, k0, radius_km;
} lp_tm_grid;
int lp_reproject_nn(const lp_latlon_grid *src_grid, const float *src, const lp_tm_grid *dst_grid,
                    float *dst, int ground_area, void *stream);

/* ---------------------------------------------------------------- batch --
 * Many independent maps (tiles, spectral bands) convolved with a few kernels:
 * the factorable-classes case of Sec. 2.2 (Eq. 4), handled map by map.  Map t
 * has ny[t] x nx[t] pixels and uses kernel psf_id[t] (0 <= psf_id < n_psf,
 * kernel p of ky[p] x kx[p]).  Each map gets the smallest padded size on each
 * axis, >= n + floor(k/2) (the bound for the input-sized window, see
 * lp_plan_set_padding), for which the library has specialised kernels; maps
 * sharing a padded size form a class, and maps of a class sharing a kernel
 * share one stored spectrum.  All host arrays are read during the call only.
 * Returns NULL on error: LP_E_INVALID (bad sizes, ids, pitch), LP_E_SIZE (no
 * specialised padded size is large enough). */
lp_batch *lp_batch_create(int n_tiles, const int64_t *ny, const int64_t *nx,
                          const int *psf_id, int n_psf, const int64_t *ky,
                          const int64_t *kx, double pitch_km);
/* As lp_batch_create, with the candidate padded lengths restricted to the
 * given lists (column axis: lengths_y, row axis: lengths_x; an empty list
 * keeps every specialised length).  Fewer, larger classes mean fewer and
 * fuller launches at the cost of more padding: the autotuner picks.  A length
 * without specialised kernels is LP_E_SIZE. */
lp_batch *lp_batch_create_padded(int n_tiles, const int64_t *ny, const int64_t *nx,
                                 const int *psf_id, int n_psf, const int64_t *ky,
                                 const int64_t *kx, double pitch_km,
                                 const int64_t *lengths_y, int n_ly,
                                 const int64_t *lengths_x, int n_lx);

/* The specialised padded lengths: axis 0 columns (Py), axis 1 rows (Px).
 * Writes up to n into out; returns how many exist. */
int lp_batch_spec_lengths(int axis, int64_t *out, int n);

void lp_batch_destroy(lp_batch *batch);
size_t lp_batch_workspace_bytes(const lp_batch *batch);

/* Caller-owned device workspace (>= lp_batch_workspace_bytes, 256-byte
 * aligned) and stream; uploads the twiddle tables and synchronises. */
int lp_batch_bind(lp_batch *batch, void *dev_ws, size_t bytes, void *stream);

/* psfs[p]: host FP64 ky[p]*kx[p] row-major kernels (Eq. 10 spectra per class,
 * as lp_kernel_spectrum).  Synchronises. */
int lp_batch_kernel_spectra(lp_batch *batch, const double *const *psfs);

/* Eq. 7 for every map of the batch (each with its own kernel; summing maps
 * of several source classes, Sec. 2.2 / Eq. 4, is lp_convolve_classes).
 * radiance[t], out[t]: device FP32 ny[t]*nx[t] per map (host array of device
 * pointers; out[t] may alias radiance[t]).  Per class and spectrum form, one
 * launch per stage covers every map (the kernels are specialised at compile
 * time for each padded length; launches merged across the classes of one
 * length ran slower than these per-class chains, which let one class's
 * column stage run beside another's row stages); the whole sequence -- three launches per class and form, forked
 * over parallel branches -- is captured once into a HIP graph and replayed
 * on the bound stream as one graph launch.  When the pointer set
 * differs from the previous call the per-map device table is re-uploaded
 * (synchronising the stream); the graph reads it and is kept. */
int lp_convolve_batched(lp_batch *batch, const float *const *radiance, float *const *out);

/* Write only rows [first, first + count) of tile `tile`'s "same" output,
 * row first at out[tile] + 0: out[tile] then holds count x nx floats.  For
 * overlap-save slabs (a slab convolved with its halo rows, only its own rows
 * kept) with no copy.  Default: all ny rows.  Takes effect at the next
 * lp_convolve_batched.  With windows, out[t] must not overlap any map's
 * radiance (the classes of a batch run one after another, so a later class
 * could read rows an earlier one already wrote).
 * Padding (Sec. 2.5): output row i sums input rows i + cy - a over the
 * kernel rows a < ky (cy = (ky - 1) / 2), so on a circle of Py rows the
 * kept rows [k0, k1) stay exact when Py >= k1 + cy and, if some kept row
 * reaches above row 0 (k0 < ky - 1 - cy), also Py >= ny + ky - 1 - cy - k0
 * (the wrapped rows must be zero padding): n + floor(k/2) for the whole
 * map, at most ny for a slab that keeps only rows whose kernel footprint
 * lies inside it (then only the first Py rows are transformed, which are
 * all the kept rows reach).  Called before the
 * first lp_batch_bind, the padding classes are chosen again from this
 * bound (lp_batch_workspace_bytes changes; per-class variants reset);
 * after it, a window that needs more rows than its map's class has is
 * refused with LP_E_STATE.  Errors: LP_E_INVALID (tile or rows out of
 * range), LP_E_SIZE (no specialised length is long enough). */
int lp_batch_set_output_rows(lp_batch *batch, int tile, int64_t first, int64_t count);

/* Graph replay (default) or direct launches (enable = 0). */
int lp_batch_use_graph(lp_batch *batch, int enable);

/* Parallel branches of the captured graph (1 to 4, default 2): the padding
 * classes use disjoint intermediates and spectra, so class g's three stages
 * are captured on branch g mod n, forked from and joined back into the
 * bound stream; the runtime may then run classes side by side.  Invalidates
 * the graph.  Errors: LP_E_INVALID. */
int lp_batch_set_graph_branches(lp_batch *batch, int n);

/* Debug mode as lp_plan_set_poison: every later lp_convolve_batched first
 * fills all the maps' intermediates with a quiet NaN (inside the captured
 * graph).  New batches take it from LP_DEBUG_POISON.  Invalidates the graph.
 * Errors: LP_E_INVALID. */
int lp_batch_set_poison(lp_batch *batch, int enable);

/* Classes: count; info for class g: {Py, Px, maps, row variants, column
 * variants, largest map row count} (up to n values); the class of map t. */
int lp_batch_group_count(const lp_batch *batch);
int lp_batch_group_info(const lp_batch *batch, int g, int64_t *info, int n);
int lp_batch_tile_group(const lp_batch *batch, int t);

/* Per-class kernel variants, as lp_plan_set_variant: LP_STAGE_ROWS selects
 * the variant of both row stages, LP_STAGE_ROWS_INVERSE the inverse row
 * stage alone, LP_STAGE_COLUMNS the column stage.  A batch computes in
 * FP32, so its variants are numbered among the plan variants without a
 * matrix-core pass (lp_batch_group_info counts the same set).  Invalidates
 * the graph.  Errors: LP_E_INVALID (class, stage or variant out of range). */
int lp_batch_set_variant(lp_batch *batch, int g, int stage, int k);
int lp_batch_get_variant(const lp_batch *batch, int g, int stage);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
