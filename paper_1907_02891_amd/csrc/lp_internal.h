// Internal declarations shared by the host plan code and the HIP kernels.
// Not part of the public ABI (include/lp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

// Largest LDS allocation one workgroup may take on gfx950 (160 KiB per CU).
constexpr int kLdsBytes = 163840;
// Largest number of complex values one thread holds during a pass.
constexpr int kEltsPerThread = 20;
constexpr int kMaxPasses = 16;

// One radix pass of a Stockham autosort transform of length n = product of
// radices.  `p` is the product of the radices of the earlier passes (the
// length of the sub-transforms already formed), `nb` = n / radix the number
// of butterflies, `tw` the offset of this pass's twiddles in the table:
// tw[tw + k*(radix-1) + (j-1)] = exp(-2 pi i j k / (p * radix)), 0<=k<p.
struct FftPass {
    int32_t radix;
    int32_t p;
    int32_t nb;
    int32_t tw;
    float inv_p;  // 1.0f / p, for the exact quotient of indices < 2^15
};

struct FftDesc {
    int32_t n;
    int32_t npass;
    int32_t split;  // radix-16 passes on MFMA: 0 none (FP32 VALU), 1 FP16 x2 terms, 2 BF16 x3 terms
    FftPass pass[kMaxPasses];
};

// Row stage arguments (forward real-to-complex with implicit zero padding,
// or inverse complex-to-real with the crop).
struct RowArgs {
    int32_t ny, nx;     // map
    int32_t m;          // half padded row length Px/2 (the complex length)
    int32_t h;          // Px/2 + 1 stored columns
    int32_t logc;       // log2 columns per block of the blocked layout
    int32_t logb;       // log2 rows per workgroup
    int32_t nblk;       // column blocks = ceil(h / 2^logc)
    FftDesc fx;         // complex transform of length m
    const float2 *tw;   // its twiddles
    const float2 *rtw;  // exp(-2 pi i k / Px), 0 <= k <= m
    const void *mf;     // matrix-core fragment table (split precision only)
};

// Column stage arguments (forward transform, spectrum multiply, inverse).
struct ColArgs {
    int32_t ny;         // stored rows of the intermediate
    int32_t py;         // padded column length
    int32_t logc;       // log2 of the column interleave C of the intermediate and spectrum
    int32_t ncols;      // columns (one per workgroup)
    int32_t ku;         // stored spectrum rows per block (py or py/2+1)
    FftDesc fy;
    const float2 *tw;
    const void *kh;     // blocked spectrum (float2 complex or float real)
    const void *mf;     // matrix-core fragment table (split precision only)
    int32_t classes;    // source classes summed before the inverse (class-sum kernels)
    int64_t w_stride;   // float2 elements from one class's intermediate to the next
    int64_t kh_stride;  // bytes from one class's spectrum to the next
};

// Size of the device-resident scratch array of lp_convolve_noalloc (one map's
// intermediate spectra), and the lookup of its address on a device (the
// current one; lp_noalloc.hip).
constexpr size_t kNoAllocBytes = size_t{128} << 20;
hipError_t noalloc_scratch(int device, void **ptr);

// Bytes of the fragment table of the split-precision radix-16 passes (both
// directions, the larger of the two split forms).
constexpr size_t kFragmentBytes = 2 * 6 * 64 * 16;

// Launchers (lp_kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_mfma_fragments(int split, void *table, hipStream_t s);
hipError_t launch_rows_r2c(const float *R, float2 *W, const RowArgs &a, int threads,
                           hipStream_t s);
hipError_t launch_cols_conv(float2 *W, const ColArgs &a, int form, bool conj_k, int threads,
                            hipStream_t s, bool class_sum = false);
hipError_t launch_rows_c2r(const float2 *W, float *S, const RowArgs &a, int threads,
                           hipStream_t s);
hipError_t launch_spec_rows(const double *K, int ky, int kx, int cx, int px, int h,
                            const double2 *tabx, double2 *t1, hipStream_t s);
// p2 > 0: the spectrum of a four-step plan, stored row r = k1 p2 + k2 holding
// frequency k1 + (py / p2) k2 (ku must then be py, in both forms).
hipError_t launch_spec_cols(const double2 *t1, int ky, int cy, int py, int ku, int h,
                            int logc, int nblk, const double2 *taby, double scale,
                            int form, void *kh, hipStream_t s, int p2 = 0);
hipError_t set_kernel_attributes();

// ------------------------------------------------ four-step column stage --
// A padded column longer than one LDS tile (Py > kMaxColLen complex values)
// is transformed as a P1 x P2 matrix: element n = P2 n1 + n2, frequency
// k = k1 + P1 k2, so that
//   X[k1 + P1 k2] = sum_n2 w_P2^(n2 k2) w_Py^(n2 k1) sum_n1 x[P2 n1 + n2] w_P1^(n1 k1),
// and the inverse runs the same steps backwards.  Three kernels:
//   outer forward   length-P1 DFTs over stride-P2 elements (rows < ny of the
//                   intermediate), times w_Py^(n2 k1), into the scratch T;
//   middle          per (column, k1): length-P2 DFT, product with the
//                   spectrum (Eq. 9), inverse length-P2 DFT, times
//                   w_Py^(-n2 k1), in place in T;
//   outer inverse   inverse length-P1 DFTs, rows n < ny back to the
//                   intermediate.
constexpr int kMaxColLen = kLdsBytes / 8;  // 20480 complex values
struct LongArgs {
    int32_t ny;          // stored rows of the intermediate
    int32_t py, p1, p2;  // Py = P1 * P2, P2 <= kMaxColLen
    int32_t lc;          // log2 of the intermediate's column interleave
    int32_t logb;        // log2 of the transforms per workgroup of the outer kernels
    FftDesc f1, f2;      // complex transforms of lengths P1 and P2
    const float2 *tw1, *tw2;
    const float2 *twq;   // exp(-2 pi i m / Py), 0 <= m < Py
    float2 *T;           // scratch: column v at T + v Py, element (k1, n2) at k1 P2 + n2
    const void *kh;      // spectrum (float real form or float2), stored row
                         // r = k1 P2 + k2 of column v at ((v >> lc) Py + r) << lc | (v & (2^lc - 1))
};
struct ColRegArgs;
// mid_spec >= 0: the middle transforms with the register kernels of column
// specialisation mid_spec (its length must be P2; tables in *mid), else the
// LDS passes of a.f2.
hipError_t launch_long_cols(float2 *W, const LongArgs &a, int ncols, int form, bool conj_k,
                            int threads_outer, int threads_mid, hipStream_t s, int mid_spec = -1,
                            const ColRegArgs *mid = nullptr);
hipError_t set_long_attributes();

}  // namespace lp

namespace lp {

// Register-resident column stage: padded column length N = R0 * R1 * R2,
// TF threads per column (one column per workgroup).
// occ: minimum waves per SIMD asked of the register allocator (0: none).
// half: the exchanges between passes go through LDS in two halves (real
// parts, then imaginary parts), which halves the exchange buffer so that
// twice as many workgroups fit on a CU; occ is then also the most waves per
// SIMD the allocator plans for (the occupancy the halved buffer allows).
// Several entries may share a length: they are the variants a plan can pick
// from (the first is the default; the autotuner measures the others).
struct ColSpec {
    int n, tf, r0, r1, r2, occ;
    int half = 0;
    // order of the pass twiddle tables (the same for every variant of a
    // length): 0: per butterfly, twiddle j of butterfly class k at
    // k (R - 1) + j - 1 (one load instruction takes several of a thread's
    // twiddles); 1: per twiddle, at (j - 1) P + k (one load instruction reads
    // a contiguous run across the lanes).  Chosen by measurement per length.
    int jmaj = 0;
    // mf: the radix-16 pass (R0 = 16: the forward's first pass, the
    // inverse's last) runs on the matrix cores with split operands; such
    // variants serve only split-precision plans, the others only FP32 plans
    int mf = 0;
};
constexpr ColSpec kColSpecs[] = {
    {5400, 360, 20, 18, 15, 5},
    {5400, 360, 20, 15, 18, 4},
    {5400, 360, 15, 18, 20, 5},
    {5400, 225, 24, 25, 9, 0},
    {4800, 320, 16, 15, 20, 5},
    {4800, 320, 20, 15, 16, 5},
    {18432, 768, 32, 24, 24, 6, 1, 1},
    {18432, 768, 32, 24, 24, 0, 0, 1},
    // split precision: radix 16 first and last (matrix cores), full exchange
    {18432, 576, 16, 32, 36, 0, 0, 1, 1},
    {18432, 576, 16, 36, 32, 0, 0, 1, 1},
    {2880, 240, 16, 12, 15, 0},
    {2880, 240, 12, 16, 15, 0},
    {512, 64, 8, 8, 8, 0},
    {1200, 120, 12, 10, 10, 0},
    {1440, 144, 12, 12, 10, 0},
    {1600, 160, 16, 10, 10, 0},
    {1920, 192, 12, 16, 10, 0},
    {1800, 180, 12, 10, 15, 0},
    {2048, 256, 16, 16, 8, 0},
    {2160, 180, 12, 12, 15, 0},
    {2592, 216, 12, 12, 18, 0},
    {3240, 270, 18, 12, 15, 0},
    {3600, 240, 16, 15, 15, 0},
    {4320, 360, 20, 18, 12, 5},
    {13500, 450, 30, 30, 15, 4, 1},
    {13500, 450, 30, 30, 15, 0},
    {13500, 450, 15, 30, 30, 4, 1},
};
constexpr int kNumColSpecs = sizeof kColSpecs / sizeof kColSpecs[0];

// Twiddle-table order of the column specialisations of length n.
constexpr bool col_jmaj(int n)
{
    for (int i = 0; i < kNumColSpecs; ++i)
        if (kColSpecs[i].n == n) return kColSpecs[i].jmaj != 0;
    return false;
}
constexpr bool col_jmaj_consistent()
{
    for (int i = 0; i < kNumColSpecs; ++i)
        if (col_jmaj(kColSpecs[i].n) != (kColSpecs[i].jmaj != 0)) return false;
    return true;
}
static_assert(col_jmaj_consistent(), "every variant of a column length shares its twiddle order");

struct ColRegArgs {
    int32_t ny;          // stored rows per column
    int32_t ku;          // stored spectrum rows per column (n or n/2+1)
    int32_t lc;          // log2 of the column interleave C of the intermediate and spectrum
    const void *kh;      // spectrum, C = 2^lc interleaved columns (float real quadrant or float2)
    int32_t classes;     // source classes summed before the inverse (class-sum kernels)
    int64_t w_stride;    // float2 elements from one class's intermediate to the next
    int64_t kh_stride;   // bytes from one class's spectrum to the next
    const float2 *tw_f1; // exp(-2 pi i j k / (R0 R1)),      k < R0,      1 <= j < R1
    const float2 *tw_f2; // exp(-2 pi i j k / N),            k < R0 R1,   1 <= j < R2
    const float2 *tw_i1; // exp(-2 pi i j k / (R2 R1)),      k < R2,      1 <= j < R1
    const float2 *tw_i2; // exp(-2 pi i j k / N),            k < R2 R1,   1 <= j < R0
    float2 *wout;        // output intermediate, same layout (nullptr: in place over the input)
    // variants whose radix-16 pass runs on the matrix cores: the split form
    // (LP_PRECISION_SPLIT_FP16 or _BF16) and its operand fragment table
    int32_t split;
    const void *mf;
};

// One map of a batched launch: the specialised kernels take a device array of
// these and read item blockIdx.y (all items of a launch share the padded
// size, the spectrum form and the twiddle tables).
struct BatchItem {
    const float *in;   // radiance, ny x nx
    float *out;        // output rows keep0 .. keep1-1 of the map, nx wide
    float2 *w;         // intermediate: (Px/2+1) columns of ny, two interleaved
    const void *kh;    // spectrum of the item's kernel at this padded size
    int32_t ny, nx;
    int32_t keep0, keep1;  // output rows [keep0, keep1) of the map, written from out[0]
};

// Index of the k-th specialisation for column length n, or -1; number of them.
int col_spec_index(int n, int k = 0);
int col_spec_count(int n);
int long_mid_spec(int n);  // specialisation for four-step middle transforms of length n (-1: none)
hipError_t launch_long_mid_reg(const LongArgs &a, const ColRegArgs &c, int idx, int ncols, int form, bool conj_k,
                               hipStream_t s);
hipError_t set_long_mid_attributes();
hipError_t launch_cols_reg(float2 *W, const ColRegArgs &a, int idx, int ncols, int form, bool conj_k,
                           hipStream_t s, const BatchItem *items = nullptr, int nitems = 1,
                           bool class_sum = false);

}  // namespace lp

namespace lp {

// Register-resident row stages: half row length M = Px/2 = R0 * R1 * R2
// (forward radix order; the inverse runs R2, R1, R0), TF threads per row,
// B rows per workgroup; pf: row tiles per workgroup (1, or 2 with the second
// tile's inputs prefetched into registers while the first is transformed; 0:
// persistent, one workgroup per resident slot looping over tiles with the
// next tile prefetched).
struct RowSpec {
    int m, tf, r0, r1, r2, b, occ, pf;
    int half = 0;  // exchanges in two halves (half the LDS); occ is then exact, pf must be 1
    // stage: the intermediate goes between HBM and the LDS in 16-byte chunks
    // (two spectrum columns of one row; the lanes of a pair cover one 32-byte
    // run of the two-column interleave), so each load or store instruction
    // touches half the cache lines of per-element accesses; full exchange,
    // one tile per workgroup
    int stage = 0;
    // mf: the radix-16 pass (R0 = 16: the forward's first pass, the
    // inverse's last) runs on the matrix cores with split operands.  Such
    // variants serve only the split-precision plans (whose form picks the
    // kernel instance), and the other variants only the FP32 plans.
    int mf = 0;
};
constexpr RowSpec kRowSpecs[] = {
    {2700, 128, 15, 15, 12, 2, 4, 1},
    {2700, 96, 12, 15, 15, 2, 3, 1},
    {2700, 192, 15, 15, 12, 2, 3, 1},
    {2700, 192, 15, 15, 12, 2, 3, 0},
    {2700, 192, 15, 15, 12, 1, 3, 0},
    {2700, 128, 15, 15, 12, 2, 3, 0},
    {2700, 180, 20, 15, 9, 2, 0, 1},
    {2700, 180, 18, 15, 10, 2, 0, 1},
    {2700, 128, 15, 15, 12, 4, 2, 1},
    {2700, 128, 15, 15, 12, 4, 2, 0},
    {2700, 128, 15, 15, 12, 6, 2, 1},
    {2700, 96, 12, 15, 15, 4, 2, 1},
    {2700, 180, 20, 15, 9, 2, 6, 1, 1},
    {2700, 128, 15, 15, 12, 2, 4, 1, 1},
    {2400, 160, 15, 16, 10, 2, 4, 1},
    {2400, 160, 16, 15, 10, 2, 4, 1},
    {6750, 256, 30, 15, 15, 2, 4, 1, 1},
    {6750, 256, 30, 15, 15, 2, 0, 1},
    {6750, 256, 30, 15, 15, 1, 4, 1, 1},
    {13500, 512, 30, 30, 15, 2, 4, 1, 1},
    {13500, 512, 30, 30, 15, 1, 4, 1, 1},
    {9216, 384, 24, 24, 16, 2, 0, 1},
    {9216, 384, 16, 24, 24, 1, 2, 1},
    {9216, 256, 16, 24, 24, 2, 2, 1},
    {9216, 384, 24, 24, 16, 1, 0, 1},
    {9216, 384, 24, 24, 16, 2, 0, 1, 0, 1},
    // the split-precision rows: radix 16 first and last, so that the forward
    // transform's first pass and the inverse's last run on the matrix cores
    // (16-36-16 keeps the paired real-to-complex pass at radix 16; 16-24-24
    // pairs radix-24 butterflies and spills at this occupancy)
    {9216, 384, 16, 36, 16, 2, 0, 1, 0, 0, 1},
    {9216, 384, 16, 36, 16, 2, 0, 1, 0, 1, 1},
    {1440, 128, 12, 12, 10, 2, 5, 1},
    {1440, 120, 15, 12, 8, 2, 0, 1},
    {1440, 128, 12, 12, 10, 2, 3, 0},
    {256, 64, 8, 8, 4, 4, 6, 1},
    {256, 64, 8, 8, 4, 4, 4, 0},
    {600, 64, 12, 10, 5, 2, 0, 1},
    {720, 96, 8, 9, 10, 2, 0, 1},
    {800, 100, 8, 10, 10, 2, 0, 1},
    {960, 120, 8, 12, 10, 2, 0, 1},
    {900, 100, 10, 9, 10, 2, 0, 1},
    {1024, 128, 8, 8, 16, 2, 0, 1},
    {1080, 120, 9, 10, 12, 2, 0, 1},
    {1296, 108, 12, 12, 9, 2, 0, 1},
    {1620, 180, 12, 9, 15, 2, 0, 1},
    {1800, 180, 12, 10, 15, 2, 0, 1},
    {2160, 180, 12, 12, 15, 2, 0, 1},
    // four and eight rows per workgroup for the shorter rows of batched tiles
    // and mid-size maps: 32- to 128-byte runs of the two-column interleave
    // (staged: through LDS in 16-byte chunks; plain: straight from registers)
    {600, 64, 12, 10, 5, 4, 0, 1, 0, 1},
    {600, 64, 12, 10, 5, 4, 0, 1},
    {600, 64, 12, 10, 5, 8, 0, 1, 0, 1},
    {600, 64, 12, 10, 5, 8, 0, 1},
    {720, 96, 8, 9, 10, 4, 0, 1, 0, 1},
    {720, 96, 8, 9, 10, 4, 0, 1},
    {720, 96, 8, 9, 10, 8, 0, 1, 0, 1},
    {720, 96, 8, 9, 10, 8, 0, 1},
    {800, 100, 8, 10, 10, 4, 0, 1, 0, 1},
    {800, 100, 8, 10, 10, 4, 0, 1},
    {800, 100, 8, 10, 10, 8, 0, 1, 0, 1},
    {800, 100, 8, 10, 10, 8, 0, 1},
    {960, 120, 8, 12, 10, 4, 0, 1, 0, 1},
    {960, 120, 8, 12, 10, 4, 0, 1},
    {960, 120, 8, 12, 10, 8, 0, 1, 0, 1},
    {960, 120, 8, 12, 10, 8, 0, 1},
    {900, 100, 10, 9, 10, 4, 0, 1, 0, 1},
    {900, 100, 10, 9, 10, 4, 0, 1},
    {900, 100, 10, 9, 10, 8, 0, 1, 0, 1},
    {900, 100, 10, 9, 10, 8, 0, 1},
    {1024, 128, 8, 8, 16, 4, 0, 1, 0, 1},
    {1024, 128, 8, 8, 16, 4, 0, 1},
    {1024, 128, 8, 8, 16, 8, 0, 1, 0, 1},
    {1024, 128, 8, 8, 16, 8, 0, 1},
    {1080, 120, 9, 10, 12, 4, 0, 1, 0, 1},
    {1080, 120, 9, 10, 12, 4, 0, 1},
    {1080, 120, 9, 10, 12, 8, 0, 1, 0, 1},
    {1080, 120, 9, 10, 12, 8, 0, 1},
    {1296, 108, 12, 12, 9, 4, 0, 1, 0, 1},
    {1296, 108, 12, 12, 9, 4, 0, 1},
    {1440, 128, 12, 12, 10, 4, 0, 1, 0, 1},
    {1440, 128, 12, 12, 10, 4, 0, 1},
    {1620, 180, 12, 9, 15, 4, 0, 1, 0, 1},
    {1620, 180, 12, 9, 15, 4, 0, 1},
    {1800, 180, 12, 10, 15, 4, 0, 1, 0, 1},
    {1800, 180, 12, 10, 15, 4, 0, 1},
    {2160, 180, 12, 12, 15, 4, 0, 1, 0, 1},
    {2160, 180, 12, 12, 15, 4, 0, 1},
};
constexpr int kNumRowSpecs = sizeof kRowSpecs / sizeof kRowSpecs[0];

struct RowRegArgs {
    int32_t ny, nx;
    int32_t lc;          // log2 of the column interleave C of the intermediate
    int32_t keep0, keep1;  // inverse: rows [keep0, keep1) are written, row r at out + (r - keep0) nx
    const float2 *rtw;   // exp(-2 pi i k / Px), 0 <= k <= M
    const float2 *tw_f1, *tw_f2, *tw_i1, *tw_i2;  // as in ColRegArgs, for length M
    // variants whose radix-16 pass runs on the matrix cores: the split form
    // (LP_PRECISION_SPLIT_FP16 or _BF16) and its operand fragment table
    int32_t split;
    const void *mf;
};

// Nearest-neighbour reprojection (lp_reproject.hip).
struct ReprojArgs {
    const float *src;        // nlat x nlon, row r at latitude lat_first - r dlat
    int64_t nlat, nlon;
    double lat_first, lon_first, dlat, dlon;  // degrees
    float *dst;              // ny x nx, row i at northing y_first - i pitch
    int64_t ny, nx;
    double x_first, y_first, pitch;           // km
    double lon0, k0, k0r;    // central meridian (degrees), central scale, k0 * R (km)
    int32_t ground_area;     // multiply by 1 / k^2 (Eq. 11)
};
hipError_t launch_reproject_nn(const ReprojArgs &a, hipStream_t s);
int64_t reproject_max_rows();

int row_spec_index(int m, int k = 0);
int row_spec_count(int m);
int row_spec_rows(int idx);
// Batched (items != nullptr): a.ny is the largest item row count, a.nx odd if
// any item's width is odd.
hipError_t launch_rows_r2c_reg(const float *R, float2 *W, const RowRegArgs &a, int idx, hipStream_t s,
                               const BatchItem *items = nullptr, int nitems = 1);
hipError_t launch_rows_c2r_reg(const float2 *W, float *S, const RowRegArgs &a, int idx, hipStream_t s,
                               const BatchItem *items = nullptr, int nitems = 1);
hipError_t set_spec_attributes();

}  // namespace lp
