// Host side of the C ABI (include/lp.h): plans, workspace layout, twiddle
// tables, the kernel spectrum and the launch sequence of the hot path.
#include "lp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lp_internal.h"

static_assert(lp::kNoAllocBytes == LP_NOALLOC_MAX_BYTES, "scratch array size");

namespace lp {
hipError_t launch_poison(void *p, size_t bytes, hipStream_t s);  // lp_debug.hip
}

namespace {

thread_local std::string g_err;
thread_local int g_status = LP_OK;

// LP_DEBUG_POISON set and not "0": new plans and batches NaN-fill their
// intermediates before every call
bool poison_default()
{
    const char *v = std::getenv("LP_DEBUG_POISON");
    return v && *v && std::strcmp(v, "0") != 0;
}

void clear_error()
{
    g_err.clear();
    g_status = LP_OK;
}

int fail(int code, const char *fmt, ...)
{
    g_status = code;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(LP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_5smooth(int64_t n)
{
    if (n <= 0) return false;
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

int64_t next_5smooth(int64_t n, bool even)
{
    for (int64_t m = std::max<int64_t>(n, 1);; ++m)
        if (is_5smooth(m) && (!even || m % 2 == 0)) return m;
}

// cos and sin of 2 pi m / n, with m reduced exactly modulo n and the angle
// folded into [0, pi/4] by octant symmetry before the FP64 evaluation, so
// that e.g. quarter turns give exact zeros.
void exp_frac(int64_t m, int64_t n, double *c, double *s)
{
    m %= n;
    if (m < 0) m += n;
    const int64_t m8 = 8 * m;
    const int64_t o = m8 / n;  // octant 0..7
    const long double pi4 = 0.785398163397448309615660845819875721L;
    long double phi;
    if (o % 2 == 0)
        phi = pi4 * static_cast<long double>(m8 - o * n) / static_cast<long double>(n);
    else
        phi = pi4 * static_cast<long double>((o + 1) * n - m8) / static_cast<long double>(n);
    const double cp = static_cast<double>(cosl(phi)), sp = static_cast<double>(sinl(phi));
    switch (o) {
        case 0: *c = cp; *s = sp; break;
        case 1: *c = sp; *s = cp; break;
        case 2: *c = -sp; *s = cp; break;
        case 3: *c = -cp; *s = sp; break;
        case 4: *c = -cp; *s = -sp; break;
        case 5: *c = -sp; *s = -cp; break;
        case 6: *c = sp; *s = -cp; break;
        default: *c = cp; *s = -sp; break;
    }
}

// Radix sequence for a 5-smooth length: as many 8s as possible (a trailing
// 2^1 or 2^2 becomes 4 or 4*4 / 2), then 5s, then 3s.
std::vector<int> radices(int64_t n, bool prefer16)
{
    int a = 0, b = 0, c = 0;
    while (n % 2 == 0) { n /= 2; ++a; }
    while (n % 3 == 0) { n /= 3; ++b; }
    while (n % 5 == 0) { n /= 5; ++c; }
    std::vector<int> r;
    if (prefer16) {
        // radix-16 passes first (matrix cores), the rest of 2^a as one pass
        for (int i = 0; i < a / 4; ++i) r.push_back(16);
        a %= 4;
        if (a > 0) r.push_back(1 << a);
        for (int i = 0; i < c; ++i) r.push_back(5);
        for (int i = 0; i < b; ++i) r.push_back(3);
        return r;
    }
    int e8 = a / 3, rem = a % 3;
    if (rem == 1 && e8 > 0) { --e8; rem = 4; }  // 8*2 -> 4*4
    for (int i = 0; i < e8; ++i) r.push_back(8);
    if (rem == 2) r.push_back(4);
    else if (rem == 4) { r.push_back(4); r.push_back(4); }
    for (int i = 0; i < c; ++i) r.push_back(5);
    for (int i = 0; i < b; ++i) r.push_back(3);
    if (rem == 1) r.push_back(2);
    return r;
}

// Pass list and FP32 twiddle table (FP64 values rounded once) of a length-n
// Stockham transform.  The table has n - 1 entries (sum of p * (r - 1)).
void make_fft(int64_t n, lp::FftDesc *d, std::vector<float> *tw, int split)
{
    std::memset(d, 0, sizeof *d);
    d->n = static_cast<int32_t>(n);
    d->split = split;
    std::vector<int> rs = radices(n, split != 0);
    // no radix-16 pass: the plain FP32 kernels (fewer registers)
    if (std::find(rs.begin(), rs.end(), 16) == rs.end()) d->split = 0;
    tw->clear();
    int64_t p = 1;
    for (size_t i = 0; i < rs.size(); ++i) {
        lp::FftPass &P = d->pass[i];
        const int r = rs[i];
        P.radix = r;
        P.p = static_cast<int32_t>(p);
        P.nb = static_cast<int32_t>(n / r);
        P.tw = static_cast<int32_t>(tw->size() / 2);
        P.inv_p = 1.0f / static_cast<float>(p);
        for (int64_t k = 0; k < p; ++k)
            for (int j = 1; j < r; ++j) {
                double c, s;
                exp_frac(j * k, p * r, &c, &s);
                tw->push_back(static_cast<float>(c));
                tw->push_back(static_cast<float>(-s));
            }
        p *= r;
    }
    d->npass = static_cast<int32_t>(rs.size());
    if (tw->empty()) { tw->push_back(1.f); tw->push_back(0.f); }
}

// Twiddles of one pass of radix r after sub-transforms of length p:
// exp(-2 pi i j k / (p r)), appended to *tw at k * (r - 1) + (j - 1), or with
// jmaj at (j - 1) * p + k (the specialised kernels give consecutive lanes
// consecutive k, so that for each j a wave reads one contiguous run).
void pass_table(int64_t p, int r, bool jmaj, std::vector<float> *tw)
{
    const size_t base = tw->size();
    tw->resize(base + 2 * static_cast<size_t>(p) * (r - 1));
    for (int64_t k = 0; k < p; ++k)
        for (int j = 1; j < r; ++j) {
            double c, s;
            exp_frac(j * k, p * r, &c, &s);
            const size_t at = jmaj ? static_cast<size_t>(j - 1) * p + k : static_cast<size_t>(k) * (r - 1) + (j - 1);
            (*tw)[base + 2 * at] = static_cast<float>(c);
            (*tw)[base + 2 * at + 1] = static_cast<float>(-s);
        }
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Complex entries of the four pass tables of a three-pass specialisation:
// forward passes (R0, R1, R2) and inverse passes (R2, R1, R0).
size_t spec_table_len(int r0, int r1, int r2)
{
    return static_cast<size_t>(r0) * (r1 - 1) + static_cast<size_t>(r0) * r1 * (r2 - 1) +
           static_cast<size_t>(r2) * (r1 - 1) + static_cast<size_t>(r2) * r1 * (r0 - 1);
}

void spec_tables(int r0, int r1, int r2, bool jmaj, std::vector<float> *tw, size_t off[4])
{
    const int tabs[4][2] = {{r0, r1}, {r0 * r1, r2}, {r2, r1}, {r2 * r1, r0}};
    tw->clear();
    for (int t = 0; t < 4; ++t) {
        off[t] = tw->size() / 2;
        pass_table(tabs[t][0], tabs[t][1], jmaj, tw);
    }
}

int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t{1} << (l + 1)) <= v) ++l;
    return l;
}

int threads_for(int64_t elems)
{
    int64_t t = (elems + 7) / 8;
    t = ((t + 63) / 64) * 64;
    return static_cast<int>(std::min<int64_t>(1024, std::max<int64_t>(64, t)));
}

}  // namespace

struct lp_plan {
    int64_t ny, nx, ky, kx;
    double pitch;
    int64_t py, px, m, h;
    // launch shape
    int logc, logb;
    int64_t nblk;
    int t_rows, t_cols;
    // transforms and tables (host copies); with four-step columns fy is the
    // length-P2 transform and f1 the length-P1 one
    lp::FftDesc fx, fy, f1;
    std::vector<float> twx, twy, rtw, tw1, twq;
    // four-step column stage (padded columns longer than one LDS tile)
    bool long_cols = false;
    int64_t p1 = 1, p2 = 0;
    int mid_spec = -1;  // column specialisation of the middle transforms (length P2), or -1
    int long_logb = 0, t_outer = 64, t_mid = 64;
    // register-resident column stage (if the padded column length has one)
    int col_spec = -1;
    int col_variant = 0, row_variant = 0;  // k-th specialisation of each length
    int row_variant_inv = 0;               // the inverse row stage's (may differ)
    size_t twc_max = 2, twr_max = 2;       // table floats reserved (largest variant)
    int variant = 0;  // 0: specialised kernels where available, 1: generic only
    int precision = LP_PRECISION_FP32;  // split forms run the generic kernels
    int classes = 1;                    // source classes summed (Eq. 4)
    size_t w_class = 0, kh_class = 0;   // bytes per class of intermediate / spectrum
    std::vector<float> twc;  // its four pass tables, concatenated
    size_t twc_off[4] = {0, 0, 0, 0};  // float2 offsets of the four tables
    // register-resident row stages (if the half row length has one)
    int row_spec = -1, row_spec_inv = -1;  // forward, inverse
    std::vector<float> twr;
    size_t twr_off[4] = {0, 0, 0, 0};
    // workspace layout (byte offsets)
    size_t off_w, off_kh, off_twx, off_twy, off_rtw, off_twc, off_twr, off_mf, bytes;
    // the column stage's output intermediate (specialised column kernels
    // write out of place; 0 bytes when the plan has none)
    size_t off_w2 = 0, w2_bytes = 0;
    size_t off_t = 0, off_tw1 = 0, off_twq = 0;  // four-step scratch and tables
    size_t scratch_bytes;
    // binding
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    int form = LP_FORM_NONE;
    // debug: NaN-fill the intermediates (and the four-step scratch) first
    bool poison = false;
    // timing: events around the stages of every timing_every-th call (0: off)
    int timing_every = 0;
    int64_t timing_seen = 0;
    std::vector<hipEvent_t> ev;
    int ev_calls = 0;
};

namespace {

constexpr int kMaxTimedCalls = 1024;

void layout(lp_plan *p)
{
    const int64_t C = int64_t{1} << p->logc;
    const size_t w = static_cast<size_t>(p->nblk) * p->ny * C * 8;
    const size_t scratch = align256(p->ky * p->kx * 8) + align256(p->ky * p->h * 16) +
                           align256(p->px * 16) + align256(p->py * 16);
    p->scratch_bytes = scratch;
    p->w_class = align256(w);
    p->kh_class = align256(static_cast<size_t>(p->nblk) * p->py * C * 8);
    p->off_w = 0;
    // a second intermediate for the specialised column kernels' output:
    // writing out of place keeps their stores off the lines that the
    // neighbouring column's workgroup is still reading (continental column
    // stage 1.036 -> 0.948 ms); four-step plans transform in place
    p->w2_bytes = (!p->long_cols && lp::col_spec_count(static_cast<int>(p->py)) > 0) ? p->w_class : 0;
    p->off_w2 = align256(std::max(p->w_class * p->classes, scratch));
    p->off_kh = p->off_w2 + p->w2_bytes;
    p->off_twx = p->off_kh + p->kh_class * p->classes;
    p->off_rtw = p->off_twx + align256(p->twx.size() * 4);
    p->off_twy = p->off_rtw + align256(p->rtw.size() * 4);
    p->off_twc = p->off_twy + align256(p->twy.size() * 4);
    p->off_twr = p->off_twc + align256(p->twc_max * 4);
    p->off_mf = p->off_twr + align256(p->twr_max * 4);
    p->bytes = p->off_mf + align256(lp::kFragmentBytes);
    if (p->long_cols) {
        // Py values per stored column for the four-step scratch, then the
        // length-P1 twiddles and exp(-2 pi i m / Py)
        p->off_t = p->bytes;
        p->off_tw1 = p->off_t + align256(static_cast<size_t>(p->nblk << p->logc) * p->py * 8);
        p->off_twq = p->off_tw1 + align256(p->tw1.size() * 4);
        p->bytes = p->off_twq + align256(p->twq.size() * 4);
    }
}

// Four-step split of a padded column longer than one LDS tile: P2 the
// longest divisor of Py that has a column specialisation (the middle
// transforms then run in registers), else the largest divisor within a tile
// (LDS passes); P1 = Py / P2 (the outer transforms, 2^logb of them per
// workgroup: about 4096 values, so that the short outer transforms still
// fill a workgroup and the reads of consecutive n2 make long runs).
void plan_long_columns(lp_plan *p)
{
    p->long_cols = p->py > lp::kMaxColLen;
    p->tw1.clear();
    p->twq.clear();
    if (!p->long_cols) {
        p->p1 = 1;
        p->p2 = 0;
        p->mid_spec = -1;
        return;
    }
    // P2: the longest divisor with a register-resident middle kernel whose
    // exchange buffer (at least 8 bytes per value) leaves room for two
    // workgroups per CU; one workgroup per CU leaves the middle transforms
    // latency-bound (27000 = 2 x 13500 ran its middle kernel 36% slower than
    // 5 x 5400)
    int64_t p2 = 1;
    p->mid_spec = -1;
    for (int64_t d = lp::kMaxColLen; d >= 2; --d) {
        if (p->py % d != 0 || p->py / d > 4096 || 2 * 8 * d > lp::kLdsBytes) continue;
        const int spec = lp::long_mid_spec(static_cast<int>(d));
        if (spec >= 0) {
            p2 = d;
            p->mid_spec = spec;
            break;
        }
    }
    if (p->mid_spec < 0)
        for (int64_t d = lp::kMaxColLen; d >= 2; --d)
            if (p->py % d == 0) { p2 = d; break; }
    p->p2 = p2;
    p->p1 = p->py / p2;
    int logb = 0;
    while ((p->p1 << (logb + 1)) <= 4096 && (int64_t{1} << (logb + 1)) <= p->p2) ++logb;
    p->long_logb = logb;
    p->t_outer = threads_for(p->p1 << logb);
    p->t_mid = threads_for(p->p2);
    make_fft(p->p1, &p->f1, &p->tw1, 0);
    make_fft(p->p2, &p->fy, &p->twy, 0);
    p->twq.resize(2 * p->py);
    for (int64_t m = 0; m < p->py; ++m) {
        double c, sn;
        exp_frac(m, p->py, &c, &sn);
        p->twq[2 * m] = static_cast<float>(c);
        p->twq[2 * m + 1] = static_cast<float>(-sn);
    }
}

// Launch shape: C = columns per workgroup of the column stage (a power of
// two whose Py*C complex values fit LDS, keeping >= min(H, 512) workgroups);
// B = rows per workgroup of the row stages ((M+1)*B complex in LDS, B*C <= 32,
// >= min(ny, 256) workgroups).
void choose_shape(lp_plan *p)
{
    // Intermediate with C = 2 interleaved columns (element i of column v at
    // ((v / 2) * ny + i) * 2 + v % 2): each row of a row-stage tile writes and
    // reads 16-byte runs instead of 8-byte ones; the column kernels take one
    // column per workgroup at stride 2.
    const int logc = p->h >= 2 ? 1 : 0;
    p->logc = logc;
    p->nblk = (p->h + (int64_t{1} << logc) - 1) >> logc;
    int logb = 0;
    for (int l = 4; l >= 0; --l) {
        const int64_t B = int64_t{1} << l;
        const int64_t groups = (p->ny + B - 1) / B;
        if ((p->m + 1) * B * 8 <= lp::kLdsBytes && groups >= std::min<int64_t>(p->ny, 256)) { logb = l; break; }
    }
    p->logb = logb;
    p->t_cols = threads_for(p->py);
    p->t_rows = threads_for(p->m << logb);
}

// Row variants of a plan: the specialisations of its half row length whose
// matrix-core flag matches the plan's precision (split-precision plans run
// only variants with the radix-16 pass on the matrix cores, FP32 plans only
// the others); variant k is the k-th of them.
int plan_row_spec(const lp_plan *p, int k)
{
    const bool split = p->precision != LP_PRECISION_FP32;
    for (int i = 0, n = lp::row_spec_count(static_cast<int>(p->m)); i < n; ++i) {
        const int idx = lp::row_spec_index(static_cast<int>(p->m), i);
        if ((lp::kRowSpecs[idx].mf != 0) == split && k-- == 0) return idx;
    }
    return -1;
}

int plan_row_count(const lp_plan *p)
{
    const bool split = p->precision != LP_PRECISION_FP32;
    int c = 0;
    for (int i = 0, n = lp::row_spec_count(static_cast<int>(p->m)); i < n; ++i)
        c += (lp::kRowSpecs[lp::row_spec_index(static_cast<int>(p->m), i)].mf != 0) == split;
    return c;
}

// Column variants of a plan, filtered the same way.
int plan_col_spec(const lp_plan *p, int k)
{
    const bool split = p->precision != LP_PRECISION_FP32;
    for (int i = 0, n = lp::col_spec_count(static_cast<int>(p->py)); i < n; ++i) {
        const int idx = lp::col_spec_index(static_cast<int>(p->py), i);
        if ((lp::kColSpecs[idx].mf != 0) == split && k-- == 0) return idx;
    }
    return -1;
}

int plan_col_count(const lp_plan *p)
{
    const bool split = p->precision != LP_PRECISION_FP32;
    int c = 0;
    for (int i = 0, n = lp::col_spec_count(static_cast<int>(p->py)); i < n; ++i)
        c += (lp::kColSpecs[lp::col_spec_index(static_cast<int>(p->py), i)].mf != 0) == split;
    return c;
}

// the row stages run specialised kernels
bool rows_specialised(const lp_plan *p)
{
    return p->variant == 0 && p->row_spec >= 0 && p->row_spec_inv >= 0;
}

void build_spec_tables(lp_plan *p)
{
    p->col_spec = plan_col_spec(p, p->col_variant);
    p->twc.clear();
    if (p->col_spec >= 0) {
        const lp::ColSpec c = lp::kColSpecs[p->col_spec];
        spec_tables(c.r0, c.r1, c.r2, c.jmaj != 0, &p->twc, p->twc_off);
    } else if (p->long_cols && p->mid_spec >= 0) {
        // the four-step middle transforms (length P2)
        const lp::ColSpec c = lp::kColSpecs[p->mid_spec];
        spec_tables(c.r0, c.r1, c.r2, c.jmaj != 0, &p->twc, p->twc_off);
    }
    // forward tables from the forward row variant, inverse ones from the
    // inverse variant, concatenated
    p->row_spec = plan_row_spec(p, p->row_variant);
    p->row_spec_inv = plan_row_spec(p, p->row_variant_inv);
    p->twr.clear();
    if (p->row_spec >= 0 && p->row_spec_inv >= 0) {
        const lp::RowSpec f = lp::kRowSpecs[p->row_spec], i = lp::kRowSpecs[p->row_spec_inv];
        size_t off_f[4], off_i[4];
        std::vector<float> ti;
        spec_tables(f.r0, f.r1, f.r2, false, &p->twr, off_f);
        spec_tables(i.r0, i.r1, i.r2, false, &ti, off_i);
        const size_t base = p->twr.size() / 2;
        p->twr.insert(p->twr.end(), ti.begin(), ti.end());
        p->twr_off[0] = off_f[0];
        p->twr_off[1] = off_f[1];
        p->twr_off[2] = base + off_i[2];
        p->twr_off[3] = base + off_i[3];
    }
}

int upload_spec_tables(lp_plan *p)
{
    hipError_t e;
    if (!p->twc.empty() &&
        (e = hipMemcpyAsync(p->ws + p->off_twc, p->twc.data(), p->twc.size() * 4, hipMemcpyHostToDevice,
                            p->stream)) != hipSuccess)
        return fail_hip(e, "twiddle upload");
    if (!p->twr.empty() &&
        (e = hipMemcpyAsync(p->ws + p->off_twr, p->twr.data(), p->twr.size() * 4, hipMemcpyHostToDevice,
                            p->stream)) != hipSuccess)
        return fail_hip(e, "twiddle upload");
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return fail_hip(e, "twiddle upload");
    return LP_OK;
}

int set_padding(lp_plan *p, int64_t py, int64_t px)
{
    // The input-sized output window needs only n + floor(k/2): a tap that
    // wraps round the padded length then always lands in the zero padding.
    if (py < p->ny + p->ky / 2 || px < p->nx + p->kx / 2)
        return fail(LP_E_SIZE, "padding %lld x %lld smaller than n + floor(k/2) = %lld x %lld",
                    (long long)py, (long long)px, (long long)(p->ny + p->ky / 2),
                    (long long)(p->nx + p->kx / 2));
    if (!is_5smooth(py) || !is_5smooth(px))
        return fail(LP_E_SIZE, "padding %lld x %lld is not of the form 2^a 3^b 5^c",
                    (long long)py, (long long)px);
    if (px % 2 != 0) return fail(LP_E_SIZE, "padded row length %lld must be even", (long long)px);
    if (py > LP_MAX_PY || px > LP_MAX_PX)
        return fail(LP_E_SIZE, "padding %lld x %lld beyond the maximum %d x %d", (long long)py,
                    (long long)px, LP_MAX_PY, LP_MAX_PX);
    p->py = py;
    p->px = px;
    p->m = px / 2;
    p->h = p->m + 1;
    if (py > lp::kMaxColLen && p->classes > 1)
        return fail(LP_E_SIZE, "padded columns of %lld (> %d) take one source class", (long long)py,
                    lp::kMaxColLen);
    make_fft(p->m, &p->fx, &p->twx, p->precision);
    make_fft(p->py, &p->fy, &p->twy, p->precision);
    plan_long_columns(p);
    p->col_variant = 0;
    p->row_variant = 0;
    p->row_variant_inv = 0;
    p->twc_max = p->twr_max = 2;
    for (int k = 0; k < lp::col_spec_count(static_cast<int>(py)); ++k) {
        const lp::ColSpec c = lp::kColSpecs[lp::col_spec_index(static_cast<int>(py), k)];
        p->twc_max = std::max<size_t>(p->twc_max, 2 * spec_table_len(c.r0, c.r1, c.r2));
    }
    if (p->mid_spec >= 0) {
        const lp::ColSpec c = lp::kColSpecs[p->mid_spec];
        p->twc_max = std::max<size_t>(p->twc_max, 2 * spec_table_len(c.r0, c.r1, c.r2));
    }
    for (int k = 0; k < lp::row_spec_count(static_cast<int>(p->m)); ++k) {
        const lp::RowSpec c = lp::kRowSpecs[lp::row_spec_index(static_cast<int>(p->m), k)];
        p->twr_max = std::max<size_t>(p->twr_max, 4 * spec_table_len(c.r0, c.r1, c.r2));  // two variants' tables
    }
    build_spec_tables(p);
    p->rtw.assign(2 * (p->m + 1), 0.f);
    for (int64_t k = 0; k <= p->m; ++k) {
        double c, s;
        exp_frac(k, p->px, &c, &s);
        p->rtw[2 * k] = static_cast<float>(c);
        p->rtw[2 * k + 1] = static_cast<float>(-s);
    }
    choose_shape(p);
    layout(p);
    return LP_OK;
}

lp::RowArgs row_args(const lp_plan *p)
{
    lp::RowArgs a{};
    a.ny = static_cast<int32_t>(p->ny);
    a.nx = static_cast<int32_t>(p->nx);
    a.m = static_cast<int32_t>(p->m);
    a.h = static_cast<int32_t>(p->h);
    a.logc = p->logc;
    a.logb = p->logb;
    a.nblk = static_cast<int32_t>(p->nblk);
    a.fx = p->fx;
    a.tw = reinterpret_cast<const float2 *>(p->ws + p->off_twx);
    a.rtw = reinterpret_cast<const float2 *>(p->ws + p->off_rtw);
    a.mf = p->ws + p->off_mf;
    return a;
}

lp::ColArgs col_args(const lp_plan *p)
{
    lp::ColArgs a{};
    a.ny = static_cast<int32_t>(p->ny);
    a.py = static_cast<int32_t>(p->py);
    a.logc = p->logc;
    a.ncols = static_cast<int32_t>(p->h);
    a.ku = static_cast<int32_t>(p->form == LP_FORM_REAL_QUADRANT ? p->py / 2 + 1 : p->py);
    a.fy = p->fy;
    a.tw = reinterpret_cast<const float2 *>(p->ws + p->off_twy);
    a.kh = p->ws + p->off_kh;
    a.mf = p->ws + p->off_mf;
    a.classes = p->classes;
    a.w_stride = static_cast<int64_t>(p->w_class / 8);
    a.kh_stride = static_cast<int64_t>(p->kh_class);
    return a;
}

bool attributes_set = false;

// The three stages.  ins: nin maps (nin = the plan's classes for a class
// sum, else 1); kh_class: the class whose spectrum a single-map call uses.
int run_path(lp_plan *p, const float *const *ins, int nin, float *out, bool adjoint, int kh_class,
             const char *who, float2 *w_scratch = nullptr)
{
    if (!p) return fail(LP_E_INVALID, "%s: null plan", who);
    if (!ins || !out) return fail(LP_E_INVALID, "%s: null data pointer", who);
    for (int t = 0; t < nin; ++t)
        if (!ins[t]) return fail(LP_E_INVALID, "%s: null data pointer", who);
    if (!p->bound) return fail(LP_E_NOMEM, "%s: no workspace bound", who);
    if (p->form == LP_FORM_NONE) return fail(LP_E_STATE, "%s: kernel spectrum not computed", who);
    const bool sum = nin > 1;
    hipError_t e;
    bool rec = false;
    if (p->timing_every > 0) {
        rec = p->timing_seen % p->timing_every == 0 && p->ev_calls < kMaxTimedCalls;
        ++p->timing_seen;
    }
    hipEvent_t *ev = rec ? &p->ev[4 * p->ev_calls] : nullptr;
    if (rec && (e = hipEventRecord(ev[0], p->stream)) != hipSuccess) return fail_hip(e, who);
    // the intermediate: the workspace's, or the scratch array given for it
    char *const wbase = w_scratch ? reinterpret_cast<char *>(w_scratch) : p->ws + p->off_w;
    float2 *W = reinterpret_cast<float2 *>(wbase);
    if (p->poison) {
        if ((e = lp::launch_poison(wbase, static_cast<size_t>(nin) * p->w_class, p->stream)) != hipSuccess ||
            (!w_scratch && (e = lp::launch_poison(p->ws + p->off_w2, p->w2_bytes, p->stream)) != hipSuccess))
            return fail_hip(e, "poison fill");
        if (p->long_cols &&
            (e = lp::launch_poison(p->ws + p->off_t, static_cast<size_t>(p->nblk << p->logc) * p->py * 8, p->stream)) !=
                hipSuccess)
            return fail_hip(e, "poison fill");
    }
    const lp::RowArgs ra = row_args(p);
    lp::ColArgs ca = col_args(p);
    ca.kh = p->ws + p->off_kh + static_cast<size_t>(kh_class) * p->kh_class;
    // the four-step middle kernels are FP32 register kernels
    const bool mid_ok = p->variant == 0 && p->precision == LP_PRECISION_FP32;
    const bool rspec = rows_specialised(p);
    lp::RowRegArgs rr{};
    if (rspec) {
        const float2 *twr = reinterpret_cast<const float2 *>(p->ws + p->off_twr);
        rr.ny = static_cast<int32_t>(p->ny);
        rr.nx = static_cast<int32_t>(p->nx);
        rr.lc = p->logc;
        rr.keep0 = 0;
        rr.keep1 = static_cast<int32_t>(p->ny);
        rr.rtw = ra.rtw;
        rr.tw_f1 = twr + p->twr_off[0];
        rr.tw_f2 = twr + p->twr_off[1];
        rr.tw_i1 = twr + p->twr_off[2];
        rr.tw_i2 = twr + p->twr_off[3];
        rr.split = p->precision;
        rr.mf = (p->precision != LP_PRECISION_FP32) ? p->ws + p->off_mf : nullptr;
    }
    for (int t = 0; t < nin; ++t) {
        float2 *Wt = reinterpret_cast<float2 *>(wbase + static_cast<size_t>(t) * p->w_class);
        e = rspec ? lp::launch_rows_r2c_reg(ins[t], Wt, rr, p->row_spec, p->stream)
                  : lp::launch_rows_r2c(ins[t], Wt, ra, p->t_rows, p->stream);
        if (e != hipSuccess) return fail_hip(e, "rows forward launch");
    }
    if (rec && (e = hipEventRecord(ev[1], p->stream)) != hipSuccess) return fail_hip(e, who);
    if (p->long_cols) {
        lp::LongArgs la{};
        la.ny = static_cast<int32_t>(p->ny);
        la.py = static_cast<int32_t>(p->py);
        la.p1 = static_cast<int32_t>(p->p1);
        la.p2 = static_cast<int32_t>(p->p2);
        la.lc = p->logc;
        la.logb = p->long_logb;
        la.f1 = p->f1;
        la.f2 = p->fy;
        la.tw1 = reinterpret_cast<const float2 *>(p->ws + p->off_tw1);
        la.tw2 = reinterpret_cast<const float2 *>(p->ws + p->off_twy);
        la.twq = reinterpret_cast<const float2 *>(p->ws + p->off_twq);
        la.T = reinterpret_cast<float2 *>(p->ws + p->off_t);
        la.kh = ca.kh;
        lp::ColRegArgs mr{};
        const float2 *twc = reinterpret_cast<const float2 *>(p->ws + p->off_twc);
        mr.tw_f1 = twc + p->twc_off[0];
        mr.tw_f2 = twc + p->twc_off[1];
        mr.tw_i1 = twc + p->twc_off[2];
        mr.tw_i2 = twc + p->twc_off[3];
        if ((e = lp::launch_long_cols(W, la, static_cast<int>(p->h), p->form, adjoint, p->t_outer, p->t_mid,
                                      p->stream, mid_ok ? p->mid_spec : -1, &mr)) != hipSuccess)
            return fail_hip(e, "four-step column stage launch");
    } else if (p->col_spec >= 0 && p->variant == 0) {
        lp::ColRegArgs cr{};
        const float2 *twc = reinterpret_cast<const float2 *>(p->ws + p->off_twc);
        cr.ny = static_cast<int32_t>(p->ny);
        cr.ku = ca.ku;
        cr.lc = p->logc;
        cr.kh = ca.kh;
        cr.classes = nin;
        cr.w_stride = ca.w_stride;
        cr.kh_stride = ca.kh_stride;
        cr.tw_f1 = twc + p->twc_off[0];
        cr.tw_f2 = twc + p->twc_off[1];
        cr.tw_i1 = twc + p->twc_off[2];
        cr.tw_i2 = twc + p->twc_off[3];
        cr.split = p->precision;
        cr.mf = (p->precision != LP_PRECISION_FP32) ? p->ws + p->off_mf : nullptr;
        // out of place into the second intermediate, which the inverse rows
        // then read (the no-allocation call has only its scratch array)
        if (!w_scratch && p->w2_bytes > 0) {
            cr.wout = reinterpret_cast<float2 *>(p->ws + p->off_w2);
            W = cr.wout;
        }
        if ((e = lp::launch_cols_reg(reinterpret_cast<float2 *>(wbase), cr, p->col_spec, static_cast<int>(p->h),
                                     p->form, adjoint, p->stream, nullptr, 1, sum)) != hipSuccess)
            return fail_hip(e, "column stage launch");
    } else {
        ca.classes = nin;
        if ((e = lp::launch_cols_conv(W, ca, p->form, adjoint, p->t_cols, p->stream, sum)) != hipSuccess)
            return fail_hip(e, "column stage launch");
    }
    if (rec && (e = hipEventRecord(ev[2], p->stream)) != hipSuccess) return fail_hip(e, who);
    e = rspec ? lp::launch_rows_c2r_reg(W, out, rr, p->row_spec_inv, p->stream)
              : lp::launch_rows_c2r(W, out, ra, p->t_rows, p->stream);
    if (e != hipSuccess) return fail_hip(e, "rows inverse launch");
    if (rec) {
        if ((e = hipEventRecord(ev[3], p->stream)) != hipSuccess) return fail_hip(e, who);
        ++p->ev_calls;
    }
    return LP_OK;
}

}  // namespace

extern "C" {

const char *lp_last_error(void) { return g_err.c_str(); }

int lp_last_status(void) { return g_status; }

const char *lp_version(void)
{
    return "lp 0.3 (gfx950, Stockham 2/3/4/5/8 FP32, radix 16 on MFMA split FP16/BF16, four-step long columns)";
}

lp_plan *lp_plan_create(int64_t ny, int64_t nx, int64_t ky, int64_t kx, double pitch_km)
{
    clear_error();
    if (ny <= 0 || nx <= 0 || ky <= 0 || kx <= 0) {
        fail(LP_E_INVALID, "sizes must be positive (ny=%lld nx=%lld ky=%lld kx=%lld)",
             (long long)ny, (long long)nx, (long long)ky, (long long)kx);
        return nullptr;
    }
    if (!(pitch_km > 0.0) || !std::isfinite(pitch_km)) {
        fail(LP_E_INVALID, "pitch must be positive and finite");
        return nullptr;
    }
    if (ny + ky / 2 > LP_MAX_PY || nx + kx / 2 > LP_MAX_PX) {
        fail(LP_E_SIZE, "n + floor(k/2) = %lld x %lld beyond the maximum %d x %d",
             (long long)(ny + ky / 2), (long long)(nx + kx / 2), LP_MAX_PY, LP_MAX_PX);
        return nullptr;
    }
    lp_plan *p = new (std::nothrow) lp_plan();
    if (!p) {
        fail(LP_E_NOMEM, "out of host memory");
        return nullptr;
    }
    p->ny = ny; p->nx = nx; p->ky = ky; p->kx = kx; p->pitch = pitch_km;
    p->poison = poison_default();
    // default: the full linear extent n + k - 1 of Sec. 2.5; where that
    // exceeds the maximum, the input-sized window's n + floor(k/2)
    int64_t py = next_5smooth(ny + ky - 1, false);
    int64_t px = next_5smooth(nx + kx - 1, true);
    if (py > LP_MAX_PY) py = next_5smooth(ny + ky / 2, false);
    if (px > LP_MAX_PX) px = next_5smooth(nx + kx / 2, true);
    if (set_padding(p, py, px) != LP_OK) {
        delete p;
        return nullptr;
    }
    return p;
}

void lp_plan_destroy(lp_plan *p)
{
    if (!p) return;
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    delete p;
}

int lp_plan_set_padding(lp_plan *p, int64_t py, int64_t px)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (p->bound) return fail(LP_E_STATE, "padding must be set before lp_plan_bind");
    return set_padding(p, py, px);
}

int lp_plan_get_padding(const lp_plan *p, int64_t *py, int64_t *px)
{
    clear_error();
    if (!p || !py || !px) return fail(LP_E_INVALID, "null argument");
    *py = p->py;
    *px = p->px;
    return LP_OK;
}

size_t lp_plan_workspace_bytes(const lp_plan *p) { return p ? p->bytes : 0; }

int lp_plan_set_kernels(lp_plan *p, int which)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (which != LP_KERNELS_AUTO && which != LP_KERNELS_GENERIC)
        return fail(LP_E_INVALID, "unknown kernel family %d", which);
    p->variant = which;
    return LP_OK;
}

int lp_plan_set_precision(lp_plan *p, int mode)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (mode != LP_PRECISION_FP32 && mode != LP_PRECISION_SPLIT_FP16 && mode != LP_PRECISION_SPLIT_BF16)
        return fail(LP_E_INVALID, "unknown precision mode %d", mode);
    if (p->bound) return fail(LP_E_STATE, "precision must be set before lp_plan_bind");
    p->precision = mode;
    // same table sizes (n - 1 twiddles per length), so the layout stands
    make_fft(p->m, &p->fx, &p->twx, mode);
    make_fft(p->py, &p->fy, &p->twy, mode);
    plan_long_columns(p);  // four-step columns stay FP32
    // the variants are those of the new precision
    p->row_variant = p->row_variant_inv = p->col_variant = 0;
    build_spec_tables(p);
    return LP_OK;
}

int lp_plan_precision(const lp_plan *p) { return p ? p->precision : -1; }

int lp_plan_kernels(const lp_plan *p)
{
    if (!p) return -1;
    if (p->variant != 0) return LP_KERNELS_GENERIC;
    const bool cols = p->col_spec >= 0;
    return (cols || rows_specialised(p)) ? LP_KERNELS_SPECIALISED : LP_KERNELS_GENERIC;
}

int lp_plan_variant_count(const lp_plan *p, int stage)
{
    if (!p) return 0;
    if (stage == LP_STAGE_ROWS || stage == LP_STAGE_ROWS_INVERSE) return plan_row_count(p);
    if (stage == LP_STAGE_COLUMNS) return plan_col_count(p);
    return 0;
}

int lp_plan_get_variant(const lp_plan *p, int stage)
{
    if (!p) return -1;
    switch (stage) {
        case LP_STAGE_ROWS: return p->row_variant;
        case LP_STAGE_COLUMNS: return p->col_variant;
        case LP_STAGE_ROWS_INVERSE: return p->row_variant_inv;
        default: return -1;
    }
}

int lp_plan_set_variant(lp_plan *p, int stage, int k)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (stage != LP_STAGE_ROWS && stage != LP_STAGE_COLUMNS && stage != LP_STAGE_ROWS_INVERSE)
        return fail(LP_E_INVALID, "unknown stage %d", stage);
    const int n = lp_plan_variant_count(p, stage);
    if (k < 0 || k >= n) return fail(LP_E_INVALID, "variant %d out of range [0, %d)", k, n);
    if (stage == LP_STAGE_COLUMNS) {
        p->col_variant = k;
    } else {
        p->row_variant_inv = k;  // LP_STAGE_ROWS sets both directions
        if (stage == LP_STAGE_ROWS) p->row_variant = k;
    }
    build_spec_tables(p);
    return p->bound ? upload_spec_tables(p) : LP_OK;
}

int lp_plan_variant_info(const lp_plan *p, int stage, int k, int *info, int n)
{
    clear_error();
    if (!p || !info) return fail(LP_E_INVALID, "null argument");
    int v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (stage == LP_STAGE_ROWS || stage == LP_STAGE_ROWS_INVERSE) {
        const int i = plan_row_spec(p, k);
        if (i < 0) return fail(LP_E_INVALID, "no row variant %d", k);
        const lp::RowSpec c = lp::kRowSpecs[i];
        const int t[11] = {c.r0, c.r1, c.r2, c.tf, c.b, c.occ, c.pf, c.m, c.half, c.stage, c.mf};
        std::copy(t, t + 11, v);
    } else if (stage == LP_STAGE_COLUMNS) {
        const int i = plan_col_spec(p, k);
        if (i < 0) return fail(LP_E_INVALID, "no column variant %d", k);
        const lp::ColSpec c = lp::kColSpecs[i];
        const int t[11] = {c.r0, c.r1, c.r2, c.tf, 1, c.occ, 1, c.n, c.half, 0, c.mf};
        std::copy(t, t + 11, v);
    } else {
        return fail(LP_E_INVALID, "unknown stage %d", stage);
    }
    for (int i = 0; i < n && i < 11; ++i) info[i] = v[i];
    return LP_OK;
}

int lp_plan_shape(const lp_plan *p, int *cols_per_group, int *rows_per_group)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (cols_per_group) *cols_per_group = 1;
    if (rows_per_group)
        *rows_per_group = rows_specialised(p) ? lp::row_spec_rows(p->row_spec) : 1 << p->logb;
    return LP_OK;
}

int lp_plan_column_split(const lp_plan *p, int64_t *p1, int64_t *p2)
{
    clear_error();
    if (!p || !p1 || !p2) return fail(LP_E_INVALID, "null argument");
    *p1 = p->long_cols ? p->p1 : 1;
    *p2 = p->long_cols ? p->p2 : p->py;
    return LP_OK;
}

int lp_plan_bind(lp_plan *p, void *ws, size_t bytes, void *stream)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (!ws) return fail(LP_E_INVALID, "null workspace");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(LP_E_INVALID, "workspace not 256-byte aligned");
    if (bytes < p->bytes)
        return fail(LP_E_NOMEM, "workspace of %zu bytes is smaller than the %zu needed", bytes, p->bytes);
    hipError_t e;
    if (!attributes_set) {
        if ((e = lp::set_kernel_attributes()) != hipSuccess || (e = lp::set_long_attributes()) != hipSuccess)
            return fail_hip(e, "kernel attributes");
        attributes_set = true;
    }
    p->ws = static_cast<char *>(ws);
    p->ws_bytes = bytes;
    p->stream = static_cast<hipStream_t>(stream);
    p->bound = false;
    p->form = LP_FORM_NONE;
    struct { size_t off; const std::vector<float> *v; } up[] = {
        {p->off_twx, &p->twx}, {p->off_rtw, &p->rtw}, {p->off_twy, &p->twy},
        {p->off_tw1, &p->tw1}, {p->off_twq, &p->twq}};
    for (auto &u : up)
        if (!u.v->empty() && (e = hipMemcpyAsync(p->ws + u.off, u.v->data(), u.v->size() * 4, hipMemcpyHostToDevice,
                                p->stream)) != hipSuccess)
            return fail_hip(e, "twiddle upload");
    const int rc = upload_spec_tables(p);
    if (rc != LP_OK) return rc;
    if (p->precision != LP_PRECISION_FP32 &&
        (e = lp::launch_mfma_fragments(p->precision, p->ws + p->off_mf, p->stream)) != hipSuccess)
        return fail_hip(e, "matrix fragment table");
    p->bound = true;
    return LP_OK;
}

namespace {

// Spectra of n kernels (classes 0 .. n-1), one storage form for all: the
// real quadrant only if every kernel is exactly mirror-symmetric on both
// axes with odd sizes (then its spectrum is real and even).
int kernel_spectra(lp_plan *p, const double *const *psfs, int n, const char *who)
{
    const int64_t ky = p->ky, kx = p->kx;
    for (int t = 0; t < n; ++t) {
        if (!psfs[t]) return fail(LP_E_INVALID, "%s: null kernel", who);
        for (int64_t i = 0; i < ky * kx; ++i)
            if (!std::isfinite(psfs[t][i]))
                return fail(LP_E_INVALID, "%s: kernel %d entry %lld is not finite", who, t, (long long)i);
    }
    if (!p->bound) return fail(LP_E_STATE, "%s before lp_plan_bind", who);
    bool sym = (ky % 2 == 1) && (kx % 2 == 1);
    for (int t = 0; sym && t < n; ++t) {
        const double *psf = psfs[t];
        for (int64_t a = 0; sym && a < ky; ++a)
            for (int64_t b = 0; b < kx; ++b) {
                const double v = psf[a * kx + b];
                if (v != psf[(ky - 1 - a) * kx + b] || v != psf[a * kx + (kx - 1 - b)]) { sym = false; break; }
            }
    }
    const int form = sym ? LP_FORM_REAL_QUADRANT : LP_FORM_COMPLEX;
    // FP64 twiddle tables exp(-2 pi i m / N)
    std::vector<double> tabx(2 * p->px), taby(2 * p->py);
    for (int64_t m = 0; m < p->px; ++m) {
        double c, s;
        exp_frac(m, p->px, &c, &s);
        tabx[2 * m] = c;
        tabx[2 * m + 1] = -s;
    }
    for (int64_t m = 0; m < p->py; ++m) {
        double c, s;
        exp_frac(m, p->py, &c, &s);
        taby[2 * m] = c;
        taby[2 * m + 1] = -s;
    }
    // scratch (overlaps the intermediate, unused until the next convolution)
    char *sc = p->ws + p->off_w;
    double *dK = reinterpret_cast<double *>(sc);
    double2 *dT1 = reinterpret_cast<double2 *>(sc + align256(ky * kx * 8));
    double2 *dTabx = reinterpret_cast<double2 *>(sc + align256(ky * kx * 8) + align256(ky * p->h * 16));
    double2 *dTaby = reinterpret_cast<double2 *>(reinterpret_cast<char *>(dTabx) + align256(p->px * 16));
    hipError_t e;
    p->form = LP_FORM_NONE;
    if ((e = hipMemcpyAsync(dTabx, tabx.data(), tabx.size() * 8, hipMemcpyHostToDevice, p->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(dTaby, taby.data(), taby.size() * 8, hipMemcpyHostToDevice, p->stream)) != hipSuccess)
        return fail_hip(e, "kernel upload");
    const int cy = static_cast<int>((ky - 1) / 2), cx = static_cast<int>((kx - 1) / 2);
    // four-step plans store every row (in the order the middle kernel reads)
    const int ku = static_cast<int>(sym && !p->long_cols ? p->py / 2 + 1 : p->py);
    const double scale = 1.0 / (static_cast<double>(p->py) * static_cast<double>(p->px));
    for (int t = 0; t < n; ++t) {
        // one kernel at a time through the scratch: the copy of kernel t+1
        // is ordered after kernel t's spectrum kernels on the stream
        if ((e = hipMemcpyAsync(dK, psfs[t], ky * kx * 8, hipMemcpyHostToDevice, p->stream)) != hipSuccess)
            return fail_hip(e, "kernel upload");
        if ((e = lp::launch_spec_rows(dK, static_cast<int>(ky), static_cast<int>(kx), cx,
                                      static_cast<int>(p->px), static_cast<int>(p->h), dTabx, dT1,
                                      p->stream)) != hipSuccess)
            return fail_hip(e, "spectrum rows launch");
        if ((e = lp::launch_spec_cols(dT1, static_cast<int>(ky), cy, static_cast<int>(p->py), ku,
                                      static_cast<int>(p->h), p->logc, static_cast<int>(p->nblk), dTaby,
                                      scale, form, p->ws + p->off_kh + static_cast<size_t>(t) * p->kh_class,
                                      p->stream, p->long_cols ? static_cast<int>(p->p2) : 0)) != hipSuccess)
            return fail_hip(e, "spectrum columns launch");
        // pageable host source: the copy may return before the transfer is
        // done, so wait before the next kernel overwrites dK
        if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return fail_hip(e, "kernel spectrum");
    }
    p->form = form;
    return LP_OK;
}

}  // namespace

int lp_kernel_spectrum(lp_plan *p, const double *psf)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (!psf) return fail(LP_E_INVALID, "null kernel");
    if (p->classes != 1)
        return fail(LP_E_STATE, "lp_kernel_spectrum on a plan of %d classes: use lp_kernel_spectra", p->classes);
    return kernel_spectra(p, &psf, 1, "lp_kernel_spectrum");
}

int lp_kernel_spectra(lp_plan *p, const double *const *psfs)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (!psfs) return fail(LP_E_INVALID, "null kernel array");
    return kernel_spectra(p, psfs, p->classes, "lp_kernel_spectra");
}

int lp_plan_spectrum_form(const lp_plan *p) { return p ? p->form : LP_FORM_NONE; }

int lp_plan_read_spectrum(lp_plan *p, float *out)
{
    clear_error();
    if (!p || !out) return fail(LP_E_INVALID, "null argument");
    if (p->form == LP_FORM_NONE) return fail(LP_E_STATE, "kernel spectrum not computed");
    const int64_t C = int64_t{1} << p->logc;
    const bool q = p->form == LP_FORM_REAL_QUADRANT;
    const int64_t ku = q ? p->py / 2 + 1 : p->py;
    const size_t elt = q ? 4 : 8;
    std::vector<float> blk(static_cast<size_t>(p->nblk) * ku * C * elt / 4);
    hipError_t e;
    if ((e = hipMemcpyAsync(blk.data(), p->ws + p->off_kh, blk.size() * 4, hipMemcpyDeviceToHost,
                            p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess)
        return fail_hip(e, "spectrum read");
    for (int64_t u = 0; u < p->py; ++u)
        for (int64_t v = 0; v < p->h; ++v) {
            const int64_t vb = v / C, c = v % C;
            float re, im;
            if (q) {
                const int64_t uq = (2 * u <= p->py) ? u : p->py - u;
                re = blk[(vb * ku + uq) * C + c];
                im = 0.f;
            } else {
                const int64_t i = ((vb * ku + u) * C + c) * 2;
                re = blk[i];
                im = blk[i + 1];
            }
            out[(u * p->h + v) * 2] = re;
            out[(u * p->h + v) * 2 + 1] = im;
        }
    return LP_OK;
}

int lp_convolve(lp_plan *p, const float *radiance, float *out)
{
    clear_error();
    if (p && p->classes != 1)
        return fail(LP_E_STATE, "lp_convolve on a plan of %d classes: use lp_convolve_classes", p->classes);
    return run_path(p, &radiance, 1, out, false, 0, "lp_convolve");
}

int lp_convolve_noalloc(lp_plan *p, const float *radiance, float *out)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "lp_convolve_noalloc: null plan");
    if (!radiance || !out) return fail(LP_E_INVALID, "lp_convolve_noalloc: null data pointer");
    if (p->classes != 1)
        return fail(LP_E_STATE, "lp_convolve_noalloc on a plan of %d classes", p->classes);
    if (p->long_cols)
        return fail(LP_E_SIZE, "lp_convolve_noalloc: padded columns of %lld take the four-step stage, "
                    "whose scratch lives in the workspace", (long long)p->py);
    if (p->w_class > LP_NOALLOC_MAX_BYTES)
        return fail(LP_E_SIZE, "lp_convolve_noalloc: the intermediate takes %zu bytes, beyond the "
                    "%zu-byte scratch array", p->w_class, static_cast<size_t>(LP_NOALLOC_MAX_BYTES));
    if (!p->bound) return fail(LP_E_NOMEM, "lp_convolve_noalloc: no workspace bound");
    if (p->form == LP_FORM_NONE) return fail(LP_E_STATE, "lp_convolve_noalloc: kernel spectrum not computed");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "lp_convolve_noalloc: current device");
    hipPointerAttribute_t attr{};
    if ((e = hipPointerGetAttributes(&attr, p->ws)) != hipSuccess)
        return fail_hip(e, "lp_convolve_noalloc: workspace attributes");
    if (attr.device != dev)
        return fail(LP_E_INVALID, "lp_convolve_noalloc: the plan's workspace is on device %d, device %d is current",
                    attr.device, dev);
    void *scratch = nullptr;
    if ((e = lp::noalloc_scratch(dev, &scratch)) != hipSuccess)
        return fail_hip(e, "lp_convolve_noalloc: scratch array address");
    return run_path(p, &radiance, 1, out, false, 0, "lp_convolve_noalloc", static_cast<float2 *>(scratch));
}

int lp_adjoint(lp_plan *p, const float *grad_out, float *grad_in)
{
    clear_error();
    if (p && p->classes != 1)
        return fail(LP_E_STATE, "lp_adjoint on a plan of %d classes: use lp_adjoint_class", p->classes);
    return run_path(p, &grad_out, 1, grad_in, true, 0, "lp_adjoint");
}

int lp_convolve_classes(lp_plan *p, const float *const *radiance, float *out)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (!radiance) return fail(LP_E_INVALID, "lp_convolve_classes: null map array");
    return run_path(p, radiance, p->classes, out, false, 0, "lp_convolve_classes");
}

int lp_adjoint_class(lp_plan *p, int cls, const float *grad_out, float *grad_in)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (cls < 0 || cls >= p->classes)
        return fail(LP_E_INVALID, "class %d outside [0, %d)", cls, p->classes);
    return run_path(p, &grad_out, 1, grad_in, true, cls, "lp_adjoint_class");
}

int lp_reproject_nn(const lp_latlon_grid *sg, const float *src, const lp_tm_grid *dg, float *dst,
                    int ground_area, void *stream)
{
    clear_error();
    if (!sg || !dg || !src || !dst) return fail(LP_E_INVALID, "lp_reproject_nn: null argument");
    if (sg->rows <= 0 || sg->cols <= 0 || dg->rows <= 0 || dg->cols <= 0)
        return fail(LP_E_INVALID, "lp_reproject_nn: grid sizes must be positive");
    const double pos[] = {sg->dlat_deg, sg->dlon_deg, dg->pitch_km, dg->k0, dg->radius_km};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v))
            return fail(LP_E_INVALID, "lp_reproject_nn: steps, pitch, k0 and radius must be positive and finite");
    const double fin[] = {sg->lat_first_deg, sg->lon_first_deg, dg->x_first_km, dg->y_first_km, dg->lon0_deg};
    for (double v : fin)
        if (!std::isfinite(v)) return fail(LP_E_INVALID, "lp_reproject_nn: grid origins must be finite");
    if (dg->rows > lp::reproject_max_rows())
        return fail(LP_E_SIZE, "lp_reproject_nn: %lld projected rows beyond the maximum %lld",
                    (long long)dg->rows, (long long)lp::reproject_max_rows());
    lp::ReprojArgs a{};
    a.src = src;
    a.nlat = sg->rows;
    a.nlon = sg->cols;
    a.lat_first = sg->lat_first_deg;
    a.lon_first = sg->lon_first_deg;
    a.dlat = sg->dlat_deg;
    a.dlon = sg->dlon_deg;
    a.dst = dst;
    a.ny = dg->rows;
    a.nx = dg->cols;
    a.x_first = dg->x_first_km;
    a.y_first = dg->y_first_km;
    a.pitch = dg->pitch_km;
    a.lon0 = dg->lon0_deg;
    a.k0 = dg->k0;
    a.k0r = dg->k0 * dg->radius_km;
    a.ground_area = ground_area != 0;
    const hipError_t e = lp::launch_reproject_nn(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "lp_reproject_nn launch");
    return LP_OK;
}

int lp_plan_set_classes(lp_plan *p, int n)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (n < 1 || n > LP_MAX_CLASSES) return fail(LP_E_INVALID, "classes %d outside [1, %d]", n, LP_MAX_CLASSES);
    if (p->bound) return fail(LP_E_STATE, "classes must be set before lp_plan_bind");
    if (n > 1 && p->long_cols)
        return fail(LP_E_SIZE, "padded columns of %lld (> %d) take one source class", (long long)p->py,
                    lp::kMaxColLen);
    p->classes = n;
    layout(p);
    return LP_OK;
}

int lp_plan_classes(const lp_plan *p) { return p ? p->classes : -1; }

int lp_plan_set_poison(lp_plan *p, int enable)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    p->poison = enable != 0;
    return LP_OK;
}

int lp_plan_timing(lp_plan *p, int enable)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    if (enable < 0) return fail(LP_E_INVALID, "timing interval %d < 0", enable);
    if (enable && p->ev.empty()) {
        p->ev.resize(4 * kMaxTimedCalls);
        for (auto &e : p->ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                p->ev.clear();
                return fail_hip(r, "event create");
            }
        }
    }
    p->timing_every = enable;
    p->timing_seen = 0;
    p->ev_calls = 0;
    return LP_OK;
}

int lp_plan_stage_ms(lp_plan *p, double *ms, int n, int *calls)
{
    clear_error();
    if (!p) return fail(LP_E_INVALID, "null plan");
    double acc[3] = {0, 0, 0};
    if (p->ev_calls > 0) {
        hipError_t e = hipEventSynchronize(p->ev[4 * p->ev_calls - 1]);
        if (e != hipSuccess) return fail_hip(e, "event sync");
        for (int c = 0; c < p->ev_calls; ++c)
            for (int s = 0; s < 3; ++s) {
                float t = 0.f;
                e = hipEventElapsedTime(&t, p->ev[4 * c + s], p->ev[4 * c + s + 1]);
                if (e != hipSuccess) return fail_hip(e, "event elapsed");
                acc[s] += t;
            }
    }
    for (int s = 0; s < n && s < 3; ++s)
        if (ms) ms[s] = acc[s];
    if (calls) *calls = p->ev_calls;
    p->ev_calls = 0;
    return LP_OK;
}

}  // extern "C"

// ====================================================================== batch
// Many maps (tiles x bands) with a few kernels (Eq. 4 applied tile by tile).
// Every map goes to a padding class (Py, Px): the smallest lengths >= n+k-1
// on each axis that have specialised kernels.  Per class and spectrum form,
// one launch per stage covers all its maps (grid.y = map), reading per-map
// pointers from a device table; spectra are shared per (class, kernel).  The
// whole launch sequence is captured once into a HIP graph and replayed.
struct lp_batch {
    struct Group {
        int64_t py = 0, px = 0, m = 0, h = 0;
        int col_variant = 0, row_variant = 0, col_spec = -1, row_spec = -1;
        int row_variant_inv = 0, row_spec_inv = -1;  // the inverse row stage's (may differ)
        std::vector<float> twc, twr, rtw;
        size_t twc_off[4] = {0, 0, 0, 0}, twr_off[4] = {0, 0, 0, 0};
        size_t twc_max = 2, twr_max = 2;
        size_t off_twc = 0, off_twr = 0, off_rtw = 0;
        std::vector<int> items;
        std::vector<int> psfs;       // distinct kernel ids used in this class
        std::vector<size_t> off_kh;  // per psfs[j]
        std::vector<int> form;       // per psfs[j]
        int64_t max_ny = 0;
        bool odd_nx = false;
        size_t off_tab[2] = {0, 0};  // BatchItem arrays: quadrant-form maps, complex-form maps
        std::vector<lp::BatchItem> tab[2];
    };
    int n = 0, n_psf = 0;
    std::vector<int64_t> ny, nx, ky, kx;
    std::vector<int64_t> keep0, keep_n;  // output rows [keep0, keep0 + keep_n) of each map
    std::vector<int64_t> ly, lx;         // padded lengths the classes may use
    std::vector<int> psf;
    double pitch = 0;
    std::vector<Group> groups;
    std::vector<int> item_group;
    std::vector<size_t> off_w;
    size_t off_scratch = 0, bytes = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false, spectra = false;
    bool use_graph = true, graph_ok = false, tables_dirty = true;
    bool poison = false;   // NaN-fill the intermediates [0, w_bytes) first
    size_t w_bytes = 0;
    hipStream_t cap = nullptr;
    // graph branches: classes are independent (own intermediates and
    // spectra), so the captured graph forks them over kBranches streams
    static constexpr int kBranches = 4;
    hipStream_t branch[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
    int branches = 2;  // measured best on the 64-tile workload (1: one linear chain)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const float *> last_in;
    std::vector<float *> last_out;
};

namespace {

std::vector<int64_t> spec_lengths(bool columns)
{
    std::vector<int64_t> v;
    if (columns) {
        for (int i = 0; i < lp::kNumColSpecs; ++i)
            if (!lp::kColSpecs[i].mf) v.push_back(lp::kColSpecs[i].n);
    } else {
        for (int i = 0; i < lp::kNumRowSpecs; ++i)
            if (!lp::kRowSpecs[i].mf) v.push_back(2 * static_cast<int64_t>(lp::kRowSpecs[i].m));
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// log2 of the column interleave of a batch's intermediates and spectra, and
// the columns (h, rounded up to whole interleave blocks) each one stores
constexpr int kBatchLogC = 1;
int64_t batch_cols(int64_t h) { return ((h + (1 << kBatchLogC) - 1) >> kBatchLogC) << kBatchLogC; }

// A batch keeps each map's intermediate and spectra in the two-column
// interleave of single-map plans (element i of column v at ((v / 2) ny + i) 2
// + v mod 2) and computes in FP32, so its row variants are those without a
// matrix-core pass: variant k of a batch is the k-th of them.
int batch_row_spec(int64_t m, int k)
{
    for (int i = 0, n = lp::row_spec_count(static_cast<int>(m)); i < n; ++i) {
        const int idx = lp::row_spec_index(static_cast<int>(m), i);
        if (lp::kRowSpecs[idx].mf == 0 && k-- == 0) return idx;
    }
    return -1;
}

// column variants of a batch: the FP32 ones
int batch_col_spec(int64_t py, int k)
{
    for (int i = 0, n = lp::col_spec_count(static_cast<int>(py)); i < n; ++i) {
        const int idx = lp::col_spec_index(static_cast<int>(py), i);
        if (lp::kColSpecs[idx].mf == 0 && k-- == 0) return idx;
    }
    return -1;
}

int batch_col_count(int64_t py)
{
    int c = 0;
    for (int i = 0, n = lp::col_spec_count(static_cast<int>(py)); i < n; ++i)
        c += lp::kColSpecs[lp::col_spec_index(static_cast<int>(py), i)].mf == 0;
    return c;
}

int batch_row_count(int64_t m)
{
    int c = 0;
    for (int i = 0, n = lp::row_spec_count(static_cast<int>(m)); i < n; ++i)
        c += lp::kRowSpecs[lp::row_spec_index(static_cast<int>(m), i)].mf == 0;
    return c;
}

void batch_group_tables(lp_batch::Group &g)
{
    g.col_spec = batch_col_spec(g.py, g.col_variant);
    g.row_spec = batch_row_spec(g.m, g.row_variant);
    g.row_spec_inv = batch_row_spec(g.m, g.row_variant_inv);
    const lp::ColSpec c = lp::kColSpecs[g.col_spec];
    spec_tables(c.r0, c.r1, c.r2, c.jmaj != 0, &g.twc, g.twc_off);
    // forward tables of the forward row variant, inverse ones of the inverse
    // variant, concatenated (as a plan's)
    const lp::RowSpec f = lp::kRowSpecs[g.row_spec], i = lp::kRowSpecs[g.row_spec_inv];
    size_t off_f[4], off_i[4];
    std::vector<float> ti;
    spec_tables(f.r0, f.r1, f.r2, false, &g.twr, off_f);
    spec_tables(i.r0, i.r1, i.r2, false, &ti, off_i);
    const size_t base = g.twr.size() / 2;
    g.twr.insert(g.twr.end(), ti.begin(), ti.end());
    g.twr_off[0] = off_f[0];
    g.twr_off[1] = off_f[1];
    g.twr_off[2] = base + off_i[2];
    g.twr_off[3] = base + off_i[3];
}

void batch_destroy_graph(lp_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ok = false;
}

int batch_upload_group_tables(lp_batch *b, lp_batch::Group &g)
{
    hipError_t e;
    if ((e = hipMemcpyAsync(b->ws + g.off_twc, g.twc.data(), g.twc.size() * 4, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(b->ws + g.off_twr, g.twr.data(), g.twr.size() * 4, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(b->ws + g.off_rtw, g.rtw.data(), g.rtw.size() * 4, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess)
        return fail_hip(e, "batch table upload");
    return LP_OK;
}

// Enqueue every launch of one batched call on stream s.
// streams[g % nstreams] carries class g (all three of its stages)
hipError_t batch_launch_all(lp_batch *b, const hipStream_t *streams, int nstreams)
{
    hipError_t e = hipSuccess;
    int gi = 0;
    for (auto &g : b->groups) {
        const hipStream_t s = streams[gi++ % nstreams];
        const float2 *twr = reinterpret_cast<const float2 *>(b->ws + g.off_twr);
        const float2 *twc = reinterpret_cast<const float2 *>(b->ws + g.off_twc);
        lp::RowRegArgs rr{};
        rr.ny = static_cast<int32_t>(g.max_ny);
        rr.nx = g.odd_nx ? 1 : 2;
        rr.lc = kBatchLogC;
        rr.rtw = reinterpret_cast<const float2 *>(b->ws + g.off_rtw);
        rr.tw_f1 = twr + g.twr_off[0];
        rr.tw_f2 = twr + g.twr_off[1];
        rr.tw_i1 = twr + g.twr_off[2];
        rr.tw_i2 = twr + g.twr_off[3];
        lp::ColRegArgs cr{};
        cr.ny = 0;
        cr.lc = kBatchLogC;
        cr.tw_f1 = twc + g.twc_off[0];
        cr.tw_f2 = twc + g.twc_off[1];
        cr.tw_i1 = twc + g.twc_off[2];
        cr.tw_i2 = twc + g.twc_off[3];
        for (int f = 0; f < 2; ++f) {
            const int nit = static_cast<int>(g.tab[f].size());
            if (nit == 0) continue;
            const lp::BatchItem *items = reinterpret_cast<const lp::BatchItem *>(b->ws + g.off_tab[f]);
            cr.ku = static_cast<int32_t>(f == 0 ? g.py / 2 + 1 : g.py);
            if ((e = lp::launch_rows_r2c_reg(nullptr, nullptr, rr, g.row_spec, s, items, nit)) != hipSuccess ||
                (e = lp::launch_cols_reg(nullptr, cr, g.col_spec, static_cast<int>(g.h), f == 0 ? 1 : 2, false,
                                         s, items, nit)) != hipSuccess ||
                (e = lp::launch_rows_c2r_reg(nullptr, nullptr, rr, g.row_spec_inv, s, items, nit)) != hipSuccess)
                return e;
        }
    }
    return e;
}

// The launch sequence under capture on b->cap: with several branches, fork
// (an event on cap that every branch stream waits for), classes round-robin
// over the branches, join (cap waits for an event on each branch), so the
// graph holds independent per-class chains.
hipError_t batch_capture_all(lp_batch *b)
{
    hipError_t e;
    if (b->poison && (e = lp::launch_poison(b->ws, b->w_bytes, b->cap)) != hipSuccess) return e;
    const int nb = std::min<int>(b->branches, static_cast<int>(b->groups.size()));
    if (nb <= 1) return batch_launch_all(b, &b->cap, 1);
    for (int i = 0; i < nb; ++i) {
        if (!b->branch[i] && (e = hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking)) != hipSuccess) return e;
        if (!b->join[i] && (e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if (!b->fork && (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventRecord(b->fork, b->cap)) != hipSuccess) return e;
    for (int i = 0; i < nb; ++i)
        if ((e = hipStreamWaitEvent(b->branch[i], b->fork, 0)) != hipSuccess) return e;
    const hipError_t le = batch_launch_all(b, b->branch, nb);
    // join every branch that joined the capture, also after a failed launch,
    // so the capture can end
    for (int i = 0; i < nb; ++i) {
        if ((e = hipEventRecord(b->join[i], b->branch[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b->cap, b->join[i], 0)) != hipSuccess) return e;
    }
    return le;
}

}  // namespace

// Padded rows a map needs for its output rows [k0, k1) (Sec. 2.5 with the
// circular wrap-round made harmless): output row i sums x[i + cy - a] over
// the kernel rows a < ky, with x = 0 outside [0, ny).  On a circle of Py
// rows the largest index k1 - 1 + cy must stay below Py (a larger one would
// wrap onto row 0).  If some kept row also reaches above row 0 (k0 + cy -
// (ky - 1) < 0), that index wraps to Py + it, which must be a zero row in
// [ny, Py): Py >= ny + ky - 1 - cy - k0.  For the whole map this is
// n + floor(k/2); for a slab that keeps only rows whose kernel footprint
// lies inside it, it is at most ny (the column stage then loads only the
// first Py rows, which are all the kept rows reach).
static int64_t batch_need_y(const lp_batch *b, int t)
{
    const int64_t k = b->ky[b->psf[t]], cy = (k - 1) / 2;
    const int64_t k0 = b->keep0[t], k1 = b->keep0[t] + b->keep_n[t];
    const int64_t top = k1 + cy;
    return (k0 + cy - (k - 1) >= 0) ? top : std::max(top, b->ny[t] + k - 1 - cy - k0);
}

// Padding classes and workspace layout from the maps, kernels, output rows
// and allowed lengths.  Host only.
static int batch_plan(lp_batch *b)
{
    const int n_tiles = b->n;
    const std::vector<int64_t> &ny = b->ny, &nx = b->nx, &ky = b->ky, &kx = b->kx, &ly = b->ly, &lx = b->lx;
    const std::vector<int> &psf_id = b->psf;
    b->groups.clear();
    b->item_group.assign(n_tiles, -1);
    for (int t = 0; t < n_tiles; ++t) {
        const int64_t need_y = batch_need_y(b, t), need_x = nx[t] + kx[psf_id[t]] / 2;
        auto py = std::lower_bound(ly.begin(), ly.end(), need_y);
        auto px = std::lower_bound(lx.begin(), lx.end(), need_x);
        if (py == ly.end() || px == lx.end())
            return fail(LP_E_SIZE, "tile %d (%lld x %lld, kernel %d) needs padding beyond the specialised sizes",
                        t, (long long)ny[t], (long long)nx[t], psf_id[t]);
        int gi = -1;
        for (size_t k = 0; k < b->groups.size(); ++k)
            if (b->groups[k].py == *py && b->groups[k].px == *px) gi = static_cast<int>(k);
        if (gi < 0) {
            lp_batch::Group g;
            g.py = *py;
            g.px = *px;
            g.m = g.px / 2;
            g.h = g.m + 1;
            for (int k = 0; k < lp::col_spec_count(static_cast<int>(g.py)); ++k) {
                const lp::ColSpec c = lp::kColSpecs[lp::col_spec_index(static_cast<int>(g.py), k)];
                g.twc_max = std::max<size_t>(g.twc_max, 2 * spec_table_len(c.r0, c.r1, c.r2));
            }
            for (int k = 0; k < lp::row_spec_count(static_cast<int>(g.m)); ++k) {
                const lp::RowSpec c = lp::kRowSpecs[lp::row_spec_index(static_cast<int>(g.m), k)];
                g.twr_max = std::max<size_t>(g.twr_max, 4 * spec_table_len(c.r0, c.r1, c.r2));  // two variants' tables
            }
            batch_group_tables(g);
            g.rtw.assign(2 * (g.m + 1), 0.f);
            for (int64_t k = 0; k <= g.m; ++k) {
                double c, s;
                exp_frac(k, g.px, &c, &s);
                g.rtw[2 * k] = static_cast<float>(c);
                g.rtw[2 * k + 1] = static_cast<float>(-s);
            }
            b->groups.push_back(std::move(g));
            gi = static_cast<int>(b->groups.size()) - 1;
        }
        lp_batch::Group &g = b->groups[gi];
        g.items.push_back(t);
        g.max_ny = std::max(g.max_ny, ny[t]);
        g.odd_nx = g.odd_nx || (nx[t] % 2 != 0);
        if (std::find(g.psfs.begin(), g.psfs.end(), psf_id[t]) == g.psfs.end()) g.psfs.push_back(psf_id[t]);
        b->item_group[t] = gi;
    }
    // workspace layout
    size_t off = 0, wtotal = 0;
    b->off_w.assign(n_tiles, 0);
    for (int t = 0; t < n_tiles; ++t) {
        const lp_batch::Group &g = b->groups[b->item_group[t]];
        b->off_w[t] = off;
        // two interleaved columns (one pad column when h is odd)
        off += align256(static_cast<size_t>(batch_cols(g.h)) * ny[t] * 8);
    }
    wtotal = off;
    b->w_bytes = wtotal;
    size_t scratch = 0;
    for (auto &g : b->groups)
        for (int p : g.psfs)
            scratch = std::max(scratch, align256(ky[p] * kx[p] * 8) + align256(ky[p] * g.h * 16) +
                                            align256(g.px * 16) + align256(g.py * 16));
    b->off_scratch = 0;  // overlaps the intermediates (idle while spectra are made)
    off = align256(std::max(wtotal, scratch));
    for (auto &g : b->groups) {
        g.off_kh.clear();
        g.form.assign(g.psfs.size(), LP_FORM_NONE);
        for (size_t j = 0; j < g.psfs.size(); ++j) {
            g.off_kh.push_back(off);
            off += align256(static_cast<size_t>(g.py) * batch_cols(g.h) * 8);
        }
        g.off_twc = off;
        off += align256(g.twc_max * 4);
        g.off_twr = off;
        off += align256(g.twr_max * 4);
        g.off_rtw = off;
        off += align256(g.rtw.size() * 4);
        for (int f = 0; f < 2; ++f) {
            g.off_tab[f] = off;
            off += align256(g.items.size() * sizeof(lp::BatchItem));
        }
    }
    b->bytes = off;
    return LP_OK;
}

extern "C" {

lp_batch *lp_batch_create(int n_tiles, const int64_t *ny, const int64_t *nx, const int *psf_id, int n_psf,
                          const int64_t *ky, const int64_t *kx, double pitch_km)
{
    return lp_batch_create_padded(n_tiles, ny, nx, psf_id, n_psf, ky, kx, pitch_km, nullptr, 0, nullptr, 0);
}

lp_batch *lp_batch_create_padded(int n_tiles, const int64_t *ny, const int64_t *nx, const int *psf_id, int n_psf,
                                 const int64_t *ky, const int64_t *kx, double pitch_km, const int64_t *lengths_y,
                                 int n_ly, const int64_t *lengths_x, int n_lx)
{
    clear_error();
    if (n_tiles <= 0 || n_psf <= 0 || !ny || !nx || !psf_id || !ky || !kx) {
        fail(LP_E_INVALID, "batch: empty or null arguments");
        return nullptr;
    }
    if (!(pitch_km > 0.0) || !std::isfinite(pitch_km)) {
        fail(LP_E_INVALID, "pitch must be positive and finite");
        return nullptr;
    }
    for (int p = 0; p < n_psf; ++p)
        if (ky[p] <= 0 || kx[p] <= 0) {
            fail(LP_E_INVALID, "kernel %d has a non-positive size", p);
            return nullptr;
        }
    std::vector<int64_t> ly = spec_lengths(true), lx = spec_lengths(false);
    if (n_ly > 0 || n_lx > 0) {
        if ((n_ly > 0 && !lengths_y) || (n_lx > 0 && !lengths_x) || n_ly < 0 || n_lx < 0) {
            fail(LP_E_INVALID, "batch: null or negative length lists");
            return nullptr;
        }
        auto restrict_to = [](std::vector<int64_t> &all, const int64_t *want, int n, const char *axis) {
            std::vector<int64_t> keep;
            for (int i = 0; i < n; ++i) {
                if (std::find(all.begin(), all.end(), want[i]) == all.end()) {
                    fail(LP_E_SIZE, "batch: %s length %lld has no specialised kernels", axis, (long long)want[i]);
                    return false;
                }
                keep.push_back(want[i]);
            }
            std::sort(keep.begin(), keep.end());
            keep.erase(std::unique(keep.begin(), keep.end()), keep.end());
            all = keep;
            return true;
        };
        if ((n_ly > 0 && !restrict_to(ly, lengths_y, n_ly, "column")) ||
            (n_lx > 0 && !restrict_to(lx, lengths_x, n_lx, "row")))
            return nullptr;
    }
    lp_batch *b = new (std::nothrow) lp_batch();
    if (!b) {
        fail(LP_E_NOMEM, "out of host memory");
        return nullptr;
    }
    b->n = n_tiles;
    b->n_psf = n_psf;
    b->poison = poison_default();
    b->pitch = pitch_km;
    b->ny.assign(ny, ny + n_tiles);
    b->keep0.assign(n_tiles, 0);
    b->keep_n.assign(ny, ny + n_tiles);
    b->nx.assign(nx, nx + n_tiles);
    b->psf.assign(psf_id, psf_id + n_tiles);
    b->ky.assign(ky, ky + n_psf);
    b->kx.assign(kx, kx + n_psf);
    b->ly = ly;
    b->lx = lx;
    for (int t = 0; t < n_tiles; ++t)
        if (ny[t] <= 0 || nx[t] <= 0 || psf_id[t] < 0 || psf_id[t] >= n_psf) {
            fail(LP_E_INVALID, "tile %d: bad size or kernel id", t);
            delete b;
            return nullptr;
        }
    if (batch_plan(b) != LP_OK) {
        delete b;
        return nullptr;
    }
    return b;
}

void lp_batch_destroy(lp_batch *b)
{
    if (!b) return;
    batch_destroy_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < lp_batch::kBranches; ++i) {
        if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

size_t lp_batch_workspace_bytes(const lp_batch *b) { return b ? b->bytes : 0; }

int lp_batch_bind(lp_batch *b, void *ws, size_t bytes, void *stream)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (!ws) return fail(LP_E_INVALID, "null workspace");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(LP_E_INVALID, "workspace not 256-byte aligned");
    if (bytes < b->bytes)
        return fail(LP_E_NOMEM, "workspace of %zu bytes is smaller than the %zu needed", bytes, b->bytes);
    hipError_t e;
    if ((e = lp::set_spec_attributes()) != hipSuccess) return fail_hip(e, "kernel attributes");
    batch_destroy_graph(b);
    b->ws = static_cast<char *>(ws);
    b->stream = static_cast<hipStream_t>(stream);
    b->bound = false;
    b->spectra = false;
    b->tables_dirty = true;
    for (auto &g : b->groups) {
        const int rc = batch_upload_group_tables(b, g);
        if (rc != LP_OK) return rc;
    }
    b->bound = true;
    return LP_OK;
}

int lp_batch_kernel_spectra(lp_batch *b, const double *const *psfs)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (!psfs) return fail(LP_E_INVALID, "null kernel array");
    for (int p = 0; p < b->n_psf; ++p) {
        if (!psfs[p]) return fail(LP_E_INVALID, "kernel %d is null", p);
        for (int64_t i = 0; i < b->ky[p] * b->kx[p]; ++i)
            if (!std::isfinite(psfs[p][i])) return fail(LP_E_INVALID, "kernel %d entry %lld is not finite", p, (long long)i);
    }
    if (!b->bound) return fail(LP_E_STATE, "lp_batch_kernel_spectra before lp_batch_bind");
    hipError_t e;
    for (auto &g : b->groups) {
        std::vector<double> tabx(2 * g.px), taby(2 * g.py);
        for (int64_t m = 0; m < g.px; ++m) {
            double c, s;
            exp_frac(m, g.px, &c, &s);
            tabx[2 * m] = c;
            tabx[2 * m + 1] = -s;
        }
        for (int64_t m = 0; m < g.py; ++m) {
            double c, s;
            exp_frac(m, g.py, &c, &s);
            taby[2 * m] = c;
            taby[2 * m + 1] = -s;
        }
        for (size_t j = 0; j < g.psfs.size(); ++j) {
            const int p = g.psfs[j];
            const int64_t ky = b->ky[p], kx = b->kx[p];
            const double *K = psfs[p];
            bool sym = (ky % 2 == 1) && (kx % 2 == 1);
            for (int64_t a = 0; sym && a < ky; ++a)
                for (int64_t c = 0; c < kx; ++c) {
                    const double v = K[a * kx + c];
                    if (v != K[(ky - 1 - a) * kx + c] || v != K[a * kx + (kx - 1 - c)]) { sym = false; break; }
                }
            char *sc = b->ws + b->off_scratch;
            double *dK = reinterpret_cast<double *>(sc);
            double2 *dT1 = reinterpret_cast<double2 *>(sc + align256(ky * kx * 8));
            double2 *dTabx = reinterpret_cast<double2 *>(sc + align256(ky * kx * 8) + align256(ky * g.h * 16));
            double2 *dTaby = reinterpret_cast<double2 *>(reinterpret_cast<char *>(dTabx) + align256(g.px * 16));
            if ((e = hipMemcpyAsync(dK, K, ky * kx * 8, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(dTabx, tabx.data(), tabx.size() * 8, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(dTaby, taby.data(), taby.size() * 8, hipMemcpyHostToDevice, b->stream)) != hipSuccess)
                return fail_hip(e, "kernel upload");
            if ((e = lp::launch_spec_rows(dK, static_cast<int>(ky), static_cast<int>(kx), static_cast<int>((kx - 1) / 2),
                                          static_cast<int>(g.px), static_cast<int>(g.h), dTabx, dT1, b->stream)) != hipSuccess)
                return fail_hip(e, "spectrum rows launch");
            const int ku = static_cast<int>(sym ? g.py / 2 + 1 : g.py);
            const double scale = 1.0 / (static_cast<double>(g.py) * static_cast<double>(g.px));
            const int form = sym ? LP_FORM_REAL_QUADRANT : LP_FORM_COMPLEX;
            if ((e = lp::launch_spec_cols(dT1, static_cast<int>(ky), static_cast<int>((ky - 1) / 2), static_cast<int>(g.py),
                                          ku, static_cast<int>(g.h), kBatchLogC,
                                          static_cast<int>(batch_cols(g.h) >> kBatchLogC), dTaby, scale, form,
                                          b->ws + g.off_kh[j], b->stream)) != hipSuccess)
                return fail_hip(e, "spectrum columns launch");
            // the scratch is reused by the next kernel: wait for this one
            if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return fail_hip(e, "kernel spectrum");
            g.form[j] = form;
        }
    }
    b->spectra = true;
    b->tables_dirty = true;
    batch_destroy_graph(b);
    return LP_OK;
}

int lp_convolve_batched(lp_batch *b, const float *const *radiance, float *const *out)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (!radiance || !out) return fail(LP_E_INVALID, "null pointer arrays");
    for (int t = 0; t < b->n; ++t)
        if (!radiance[t] || !out[t]) return fail(LP_E_INVALID, "tile %d: null data pointer", t);
    if (!b->bound) return fail(LP_E_NOMEM, "no workspace bound");
    if (!b->spectra) return fail(LP_E_STATE, "kernel spectra not computed");
    hipError_t e;
    bool changed = b->tables_dirty || b->last_in.size() != static_cast<size_t>(b->n);
    for (int t = 0; !changed && t < b->n; ++t) changed = b->last_in[t] != radiance[t] || b->last_out[t] != out[t];
    if (changed) {
        for (auto &g : b->groups) {
            g.tab[0].clear();
            g.tab[1].clear();
            for (int t : g.items) {
                const size_t j = std::find(g.psfs.begin(), g.psfs.end(), b->psf[t]) - g.psfs.begin();
                lp::BatchItem it{};
                it.in = radiance[t];
                it.out = out[t];
                it.w = reinterpret_cast<float2 *>(b->ws + b->off_w[t]);
                it.kh = b->ws + g.off_kh[j];
                it.ny = static_cast<int32_t>(b->ny[t]);
                it.nx = static_cast<int32_t>(b->nx[t]);
                it.keep0 = static_cast<int32_t>(b->keep0[t]);
                it.keep1 = static_cast<int32_t>(b->keep0[t] + b->keep_n[t]);
                g.tab[g.form[j] == LP_FORM_REAL_QUADRANT ? 0 : 1].push_back(it);
            }
            for (int f = 0; f < 2; ++f)
                if (!g.tab[f].empty() &&
                    (e = hipMemcpyAsync(b->ws + g.off_tab[f], g.tab[f].data(), g.tab[f].size() * sizeof(lp::BatchItem),
                                        hipMemcpyHostToDevice, b->stream)) != hipSuccess)
                    return fail_hip(e, "batch table upload");
        }
        if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return fail_hip(e, "batch table upload");
        // the launch grids depend on the per-form split: rebuild the graph
        if (b->tables_dirty) batch_destroy_graph(b);
        b->last_in.assign(radiance, radiance + b->n);
        b->last_out.assign(out, out + b->n);
        b->tables_dirty = false;
    }
    if (!b->use_graph) {
        if (b->poison && (e = lp::launch_poison(b->ws, b->w_bytes, b->stream)) != hipSuccess)
            return fail_hip(e, "poison fill");
        if ((e = batch_launch_all(b, &b->stream, 1)) != hipSuccess) return fail_hip(e, "batched launch");
        return LP_OK;
    }
    if (!b->graph_ok) {
        if (!b->cap && (e = hipStreamCreate(&b->cap)) != hipSuccess) return fail_hip(e, "capture stream");
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return fail_hip(e, "graph capture");
        const hipError_t le = batch_capture_all(b);
        hipGraph_t gph = nullptr;
        e = hipStreamEndCapture(b->cap, &gph);
        if (le != hipSuccess) {
            if (gph) (void)hipGraphDestroy(gph);
            return fail_hip(le, "batched launch (capture)");
        }
        if (e != hipSuccess) return fail_hip(e, "graph capture");
        b->graph = gph;
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
            batch_destroy_graph(b);
            return fail_hip(e, "graph instantiate");
        }
        b->graph_ok = true;
    }
    if ((e = hipGraphLaunch(b->exec, b->stream)) != hipSuccess) return fail_hip(e, "graph launch");
    return LP_OK;
}

int lp_batch_set_output_rows(lp_batch *b, int tile, int64_t first, int64_t count)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (tile < 0 || tile >= b->n) return fail(LP_E_INVALID, "tile %d outside [0, %d)", tile, b->n);
    if (first < 0 || count < 1 || first + count > b->ny[tile])
        return fail(LP_E_INVALID, "tile %d: rows [%lld, %lld) outside [0, %lld)", tile, (long long)first,
                    (long long)(first + count), (long long)b->ny[tile]);
    if (b->keep0[tile] == first && b->keep_n[tile] == count) return LP_OK;
    const int64_t k0 = b->keep0[tile], kn = b->keep_n[tile];
    b->keep0[tile] = first;
    b->keep_n[tile] = count;
    if (!b->bound && !b->ws) {
        // before the first bind: the padding classes follow the windows
        const int rc = batch_plan(b);
        if (rc != LP_OK) {
            b->keep0[tile] = k0;
            b->keep_n[tile] = kn;
            (void)batch_plan(b);
            return rc;
        }
    } else if (batch_need_y(b, tile) > b->groups[b->item_group[tile]].py) {
        const int64_t need = batch_need_y(b, tile);
        b->keep0[tile] = k0;
        b->keep_n[tile] = kn;
        return fail(LP_E_STATE, "tile %d: rows [%lld, %lld) need %lld padded rows, more than its class's %lld; "
                    "set such windows before lp_batch_bind", tile, (long long)first, (long long)(first + count),
                    (long long)need, (long long)b->groups[b->item_group[tile]].py);
    }
    b->tables_dirty = true;
    return LP_OK;
}

int lp_batch_spec_lengths(int axis, int64_t *out, int n)
{
    const std::vector<int64_t> v = spec_lengths(axis == 0);
    for (int i = 0; i < n && i < static_cast<int>(v.size()); ++i) out[i] = v[i];
    return static_cast<int>(v.size());
}

int lp_batch_use_graph(lp_batch *b, int enable)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    b->use_graph = enable != 0;
    return LP_OK;
}

int lp_batch_set_graph_branches(lp_batch *b, int n)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (n < 1 || n > lp_batch::kBranches)
        return fail(LP_E_INVALID, "graph branches %d outside [1, %d]", n, lp_batch::kBranches);
    if (b->branches != n) {
        b->branches = n;
        batch_destroy_graph(b);
        b->graph_ok = false;
    }
    return LP_OK;
}

int lp_batch_set_poison(lp_batch *b, int enable)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (b->poison != (enable != 0)) {
        b->poison = enable != 0;
        batch_destroy_graph(b);
    }
    return LP_OK;
}

int lp_batch_group_count(const lp_batch *b) { return b ? static_cast<int>(b->groups.size()) : 0; }

int lp_batch_group_info(const lp_batch *b, int g, int64_t *info, int n)
{
    clear_error();
    if (!b || !info) return fail(LP_E_INVALID, "null argument");
    if (g < 0 || g >= static_cast<int>(b->groups.size())) return fail(LP_E_INVALID, "no group %d", g);
    const lp_batch::Group &gr = b->groups[g];
    const int64_t v[6] = {gr.py, gr.px, static_cast<int64_t>(gr.items.size()),
                          batch_row_count(gr.m), batch_col_count(gr.py),
                          gr.max_ny};
    for (int i = 0; i < n && i < 6; ++i) info[i] = v[i];
    return LP_OK;
}

int lp_batch_tile_group(const lp_batch *b, int t) { return (b && t >= 0 && t < b->n) ? b->item_group[t] : -1; }

int lp_batch_set_variant(lp_batch *b, int g, int stage, int k)
{
    clear_error();
    if (!b) return fail(LP_E_INVALID, "null batch");
    if (g < 0 || g >= static_cast<int>(b->groups.size())) return fail(LP_E_INVALID, "no group %d", g);
    lp_batch::Group &gr = b->groups[g];
    if (stage == LP_STAGE_ROWS || stage == LP_STAGE_ROWS_INVERSE) {
        if (k < 0 || k >= batch_row_count(gr.m)) return fail(LP_E_INVALID, "no row variant %d", k);
        if (stage == LP_STAGE_ROWS) gr.row_variant = k;
        gr.row_variant_inv = k;
    } else if (stage == LP_STAGE_COLUMNS) {
        if (k < 0 || k >= batch_col_count(gr.py)) return fail(LP_E_INVALID, "no column variant %d", k);
        gr.col_variant = k;
    } else {
        return fail(LP_E_INVALID, "unknown stage %d", stage);
    }
    batch_group_tables(gr);
    batch_destroy_graph(b);
    return b->bound ? batch_upload_group_tables(b, gr) : LP_OK;
}

int lp_batch_get_variant(const lp_batch *b, int g, int stage)
{
    if (!b || g < 0 || g >= static_cast<int>(b->groups.size())) return -1;
    return stage == LP_STAGE_ROWS             ? b->groups[g].row_variant
           : stage == LP_STAGE_ROWS_INVERSE ? b->groups[g].row_variant_inv
           : stage == LP_STAGE_COLUMNS      ? b->groups[g].col_variant
                                            : -1;
}

}  // extern "C"
