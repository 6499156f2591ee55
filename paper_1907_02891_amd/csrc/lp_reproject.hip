// Nearest-neighbour reprojection of a longitude-latitude (plate carree)
// radiance map onto a transverse Mercator grid (Sec. 2.4), with the scale
// factor of Eq. 11 for the optional ground-area weight.
//
// Each projected pixel centre (x, y) (km from the central meridian and the
// equator) is mapped back to latitude and longitude with the spherical
// inverse transverse Mercator of Snyder (the paper's reference for Eq. 11):
//   D = y / (k0 R),  phi = asin(sin D / cosh(x / (k0 R))),
//   lambda = lambda0 + atan2(sinh(x / (k0 R)), cos D),
// then takes the source pixel nearest in (row, column) index space (halves
// to even), or 0 outside the source grid.  The ground-area weight is 1 / k^2
// with k = k0 cosh(x / (k0 R)) (Eq. 11): the projection is conformal, so a
// projected cell of pitch^2 covers pitch^2 / k^2 of ground.
//
// A workgroup covers 4 rows x 64 columns of the projected grid: the row terms
// (sin D, cos D) and the column terms (sinh, cosh of x / (k0 R), 1 / k^2) are
// computed once per workgroup into LDS, so each pixel pays one asin and one
// atan2.  FP64 throughout, with no contraction of multiply-adds, so that the
// index a pixel rounds to is decided by the same arithmetic as a plain
// evaluation of the formulas.
#include <hip/hip_runtime.h>

#include "lp_internal.h"

namespace lp {

namespace {

constexpr int kRowsPerGroup = 4, kColsPerGroup = 64;

__global__ void __launch_bounds__(kRowsPerGroup * kColsPerGroup) k_reproject_nn(ReprojArgs a)
{
#pragma clang fp contract(off)
    __shared__ double2 rowt[kRowsPerGroup];  // sin D, cos D
    __shared__ double colt[kColsPerGroup][3];  // sinh xs, cosh xs, 1 / k^2
    const int t = threadIdx.x;
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * kRowsPerGroup;
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kColsPerGroup;
    if (t < kColsPerGroup) {
        const double x = a.x_first + a.pitch * static_cast<double>(j0 + t);
        const double xs = x / a.k0r;
        const double ch = cosh(xs);
        const double k = a.k0 * ch;
        colt[t][0] = sinh(xs);
        colt[t][1] = ch;
        colt[t][2] = 1.0 / (k * k);
    } else if (t < kColsPerGroup + kRowsPerGroup) {
        const double y = a.y_first - a.pitch * static_cast<double>(i0 + (t - kColsPerGroup));
        const double D = y / a.k0r;
        rowt[t - kColsPerGroup] = make_double2(sin(D), cos(D));
    }
    __syncthreads();
    const int r = t / kColsPerGroup, c = t % kColsPerGroup;
    const int64_t i = i0 + r, j = j0 + c;
    if (i >= a.ny || j >= a.nx) return;
    const double deg = M_PI / 180.0;
    const double2 rd = rowt[r];
    const double phi = asin(rd.x / colt[c][1]);
    const double lam = a.lon0 * deg + atan2(colt[c][0], rd.y);
    const double rowf = (a.lat_first - phi / deg) / a.dlat;
    const double colf = (lam / deg - a.lon_first) / a.dlon;
    const double rr = rint(rowf), cc = rint(colf);
    float v = 0.f;
    if (rr >= 0.0 && rr < static_cast<double>(a.nlat) && cc >= 0.0 && cc < static_cast<double>(a.nlon)) {
        v = a.src[static_cast<int64_t>(rr) * a.nlon + static_cast<int64_t>(cc)];
        if (a.ground_area) v = static_cast<float>(static_cast<double>(v) * colt[c][2]);
    }
    a.dst[i * a.nx + j] = v;
}

}  // namespace

hipError_t launch_reproject_nn(const ReprojArgs &a, hipStream_t s)
{
    const dim3 g(static_cast<unsigned>((a.nx + kColsPerGroup - 1) / kColsPerGroup),
                 static_cast<unsigned>((a.ny + kRowsPerGroup - 1) / kRowsPerGroup));
    hipLaunchKernelGGL(k_reproject_nn, g, dim3(kRowsPerGroup * kColsPerGroup), 0, s, a);
    return hipGetLastError();
}

int64_t reproject_max_rows() { return int64_t{65535} * kRowsPerGroup; }

}  // namespace lp
