// cde_api.hip -- host side of the C ABI declared in include/cde.h: argument
// validation, per-setting coefficient preparation in FP64, device memory of
// the model, and stream-ordered kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cde_common.h"
#include "cde_kernels.h"

using namespace cde;

// Radial Epanechnikov setting (Section 4's kernel in the scaled form of
// Section 2): K_h(t) = c_d / prod h * max(0, 1 - |t/h|^2), c_d = (d+2)/(2 V_d).
double cde::log_epan_norm(const double* h, int d)
{
    const double log_vd = 0.5 * d * std::log(3.14159265358979323846) - std::lgamma(0.5 * d + 1.0);
    double s = std::log((d + 2.0) / 2.0) - log_vd;
    for (int k = 0; k < d; ++k) s -= std::log(h[k]);
    return s;
}

namespace {

thread_local std::string g_last_error;

cde_status fail(cde_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

cde_status hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? CDE_ENOMEM : CDE_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

bool supported_dims(int dx, int dy)
{
    return (dy == 1 || dy == 2) && ((dx >= 1 && dx <= 8) || dx == 16);
}

bool valid_bandwidths(const double* h, int k)
{
    if (!h) return false;
    for (int q = 0; q < k; ++q)
        if (!(h[q] > 0.0) || !std::isfinite(h[q])) return false;
    return true;
}

// Representable range of a Gaussian setting for a model of precision p, over
// data whose per-dimension extents (max - min) are `range`.  With c_k =
// log2(e) / (2 h_k^2), X = sum_{k < dx} range_k^2 c_k and Y the same over the
// y dimensions (the largest exponents any pair can have):
//   - every pass: each c_k <= CMAX (c_k, and the excluded-pair sentinel 1e20
//     times it, stay finite in FP32 for FP32 models), X <= SMAX and
//     Y <= SMAX (no pair's exponent overflows);
//   - the diagonal pass (per-dimension bandwidths: values, gradients, the
//     LOO part of the ISE, and every grid of an FP64 model) forms exponents
//     in the model's precision relative to a per-point reference, so its
//     absolute rounding error grows with the exponents' size, about
//     (dx + dy + 2) (X + Y) u; (X + Y)(dx + dy + 2) <= DMAX keeps that far
//     below the 2^64 (FP64: 2^640) headroom of its sums, so no sum
//     overflows.  (The grid and query passes form shifted exponents in FP64
//     and need only the first rule.)
// Outside these ranges the kernels would produce inf - inf or 0 * inf.
constexpr double CMAX_F32 = 0x1p59, SMAX_F32 = 0x1p100, DMAX_F32 = 0x1p29;
constexpr double CMAX_F64 = 0x1p900, SMAX_F64 = 0x1p900, DMAX_F64 = 0x1p61;

// Largest exponent of one group of dimensions; h_step = 0 broadcasts h[0].
double group_exponent(const double* range, int cnt, const double* h, int h_step, double* cmax)
{
    double s = 0.0, cm = 0.0;
    for (int k = 0; k < cnt; ++k) {
        const double hk = h[k * h_step];
        const double c = LOG2E / (2.0 * hk * hk);
        cm = std::max(cm, c);
        s += range[k] * range[k] * c;
    }
    *cmax = cm;
    return s;
}

cde_status check_group(const double* range, int cnt, const double* h, int h_step, cde_precision p,
                       const char* who, const char* axis, double* exponent)
{
    double cm = 0.0;
    const double e = group_exponent(range, cnt, h, h_step, &cm);
    if (exponent) *exponent = e;
    const double cmax = p == CDE_F64 ? CMAX_F64 : CMAX_F32, smax = p == CDE_F64 ? SMAX_F64 : SMAX_F32;
    if (cm <= cmax && e <= smax) return CDE_OK;
    char msg[320];
    std::snprintf(msg, sizeof msg,
                  "%s: %s bandwidth too small for the kernels' %s arithmetic on this data "
                  "(needs log2(e)/(2h^2) <= 2^%d and sum_k range_k^2 log2(e)/(2h_k^2) <= 2^%d; "
                  "got %.3g and %.3g)",
                  who, axis, p == CDE_F64 ? "FP64" : "FP32", p == CDE_F64 ? 900 : 59,
                  p == CDE_F64 ? 900 : 100, cm, e);
    return fail(CDE_EUNSUPPORTED, msg);
}

// The diagonal pass's extra rule on the exponents X and Y of one setting.
cde_status check_diag_pass(double ex, double ey, int dx, int dy, cde_precision p, const char* who)
{
    const double lim = p == CDE_F64 ? DMAX_F64 : DMAX_F32;
    const double v = (ex + ey) * (dx + dy + 2);
    if (v <= lim) return CDE_OK;
    char msg[320];
    std::snprintf(msg, sizeof msg,
                  "%s: bandwidths too small for the diagonal pass's %s exponents on this data "
                  "(needs (X + Y)(dx + dy + 2) <= 2^%d with X, Y = sum_k range_k^2 log2(e)/(2h_k^2) "
                  "over the x and the y dimensions; got %.3g)",
                  who, p == CDE_F64 ? "FP64" : "FP32", p == CDE_F64 ? 61 : 29, v);
    return fail(CDE_EUNSUPPORTED, msg);
}

// One diagonal setting h [dx + dy] against the extents `range` [dx + dy];
// `diag`: the setting runs on the diagonal pass.
cde_status check_setting(const double* range, int dx, int dy, const double* h, cde_precision p,
                         bool diag, const char* who)
{
    double ex = 0.0, ey = 0.0;
    cde_status st = check_group(range, dx, h, 1, p, who, "x", &ex);
    if (st != CDE_OK) return st;
    st = check_group(range + dx, dy, h + dx, 1, p, who, "y", &ey);
    if (st != CDE_OK || !diag) return st;
    return check_diag_pass(ex, ey, dx, dy, p, who);
}

unsigned long long decode_ordered(unsigned long long u)
{
    return (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
}

// The model's data extent, computed by cde_create; the first call waits for
// its device-to-host copy.
cde_status ensure_extent(cde_model* m, const char* who)
{
    if (!m->ext_known) {
        hipError_t e = hipEventSynchronize(m->ext_event);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(data extent)");
        const int d = m->dx + m->dy;
        for (int c = 0; c < d; ++c) {
            const unsigned long long lo = decode_ordered(m->ext_host[2 * c]);
            const unsigned long long hi = decode_ordered(m->ext_host[2 * c + 1]);
            double a, b;
            std::memcpy(&a, &lo, sizeof a);
            std::memcpy(&b, &hi, sizeof b);
            m->range[c] = b - a;
        }
        m->data_finite = m->ext_host[2 * MAXP] == 0;
        m->ext_known = true;
    }
    if (!m->data_finite)
        return fail(CDE_EINVAL, std::string(who) + ": the training data hold non-finite values");
    return CDE_OK;
}

// Bandwidth checks of the model calls: finite and > 0 (CDE_EINVAL), then
// within the representable range for the model's data and the pass that
// runs the call (CDE_EUNSUPPORTED).
cde_status check_model_settings(cde_model* m, const double* h, int g, bool diag, const char* who)
{
    const int p = m->dx + m->dy;
    if (!valid_bandwidths(h, g * p))
        return fail(CDE_EINVAL, std::string(who) + ": bandwidths must be finite and > 0");
    cde_status st = ensure_extent(m, who);
    if (st != CDE_OK) return st;
    for (int s = 0; s < g; ++s) {
        st = check_setting(m->range, m->dx, m->dy, h + (size_t)s * p, m->prec, diag, who);
        if (st != CDE_OK) return st;
    }
    return CDE_OK;
}

cde_status check_model_grid(cde_model* m, const double* hx, int n_hx, const double* hy, int n_hy,
                            bool diag, const char* who)
{
    if (!valid_bandwidths(hx, n_hx) || !valid_bandwidths(hy, n_hy))
        return fail(CDE_EINVAL, std::string(who) + ": bandwidths must be finite and > 0");
    cde_status st = ensure_extent(m, who);
    if (st != CDE_OK) return st;
    double exmax = 0.0, eymax = 0.0, e = 0.0;
    for (int a = 0; a < n_hx; ++a) {
        if ((st = check_group(m->range, m->dx, hx + a, 0, m->prec, who, "x", &e)) != CDE_OK) return st;
        exmax = std::max(exmax, e);
    }
    for (int b = 0; b < n_hy; ++b) {
        if ((st = check_group(m->range + m->dx, m->dy, hy + b, 0, m->prec, who, "y", &e)) != CDE_OK)
            return st;
        eymax = std::max(eymax, e);
    }
    return diag ? check_diag_pass(exmax, eymax, m->dx, m->dy, m->prec, who) : CDE_OK;
}

// Device bytes of a model's packed rows plus the extent record in their tail.
constexpr size_t EXT_BYTES = 512;
size_t packed_bytes(int64_t npad, int stride, size_t elt)
{
    return ((size_t)npad * stride * elt + 255) / 256 * 256 + EXT_BYTES;
}

// Gaussian coefficients of one diagonal setting (Section 2: K_h(t) =
// h^{-d} K(t/h), K the standard normal density).
template <typename T>
void fill_set(DiagSet<T>& s, const double* h, int dx, int dy)
{
    std::memset(&s, 0, sizeof s);
    double lcx = 0.0, lcy = 0.0;
    for (int k = 0; k < dx + dy; ++k) {
        s.c[k] = (T)(LOG2E / (2.0 * h[k] * h[k]));
        s.inv_h[k] = 1.0 / h[k];
        s.inv_h3[k] = 1.0 / (h[k] * h[k] * h[k]);
        if (k < dx) lcx -= std::log(h[k]) + HALF_LOG_2PI;
        else lcy -= std::log(h[k]) + HALF_LOG_2PI;
    }
    s.log_cx = lcx;
    s.log_cy = lcy;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

size_t round_scratch(size_t bytes) { return (bytes + 4095) & ~size_t(4095); }

cde_status ensure_scratch(cde_model* m, size_t bytes)
{
    if (m->scratch_bytes >= bytes) return CDE_OK;
    if (m->scratch) {
        hipError_t e = hipFree(m->scratch);  // device-synchronising: no call still uses it
        m->scratch = nullptr;
        m->bytes -= m->scratch_bytes;
        m->scratch_bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree(scratch)");
    }
    bytes = round_scratch(bytes);
    hipError_t e = hipMalloc(&m->scratch, bytes);
    if (e != hipSuccess) {
        m->scratch = nullptr;
        return hip_fail(e, "hipMalloc(scratch)");
    }
    m->scratch_bytes = bytes;
    m->bytes += bytes;
    return CDE_OK;
}

// A grouped grid evaluation keeps its state in the model's scratch between
// cde_launch_batch calls; no other call may use the scratch meanwhile.
cde_status reject_if_batching(const cde_model* m, const char* who)
{
    if (m->batch_next == 0) return CDE_OK;
    return fail(CDE_EINVAL, std::string(who) +
                                ": the model is in the middle of a grouped grid evaluation "
                                "(cde_launch_batch ranges up to its last point are still to come)");
}

// FNV-1a signature of a grid and criterion (detects a change between the
// ranges of one grouped evaluation).
uint64_t grid_signature(const double* hx, int n_hx, const double* hy, int n_hy, int crit)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t bytes) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t k = 0; k < bytes; ++k) h = (h ^ c[k]) * 1099511628211ull;
    };
    mix(&n_hx, sizeof n_hx);
    mix(hx, sizeof(double) * n_hx);
    mix(&n_hy, sizeof n_hy);
    mix(hy, sizeof(double) * n_hy);
    mix(&crit, sizeof crit);
    return h;
}

// Value (and gradient) for a list of diagonal settings, reduced into
// totals[g] (and grad[g][dx+dy]); per-setting non-finite counts are summed
// into *nonfinite when given.
// Scratch of a list/gradient call over g settings: block rows and counts,
// then the chunk partials of one launch.
template <typename T>
size_t diag_list_scratch(const cde_model* m, int g, bool grad, int* chunks_out)
{
    const int nblocks = (int)(m->npad / TILE);
    const int nv = grad ? m->dx + m->dy + 2 : 2;
    const int per_launch = std::min(g, MAX_SETS_PER_LAUNCH);
    const int chunks = diag_chunks<T>(m, per_launch, grad, MAX_DIAG_PARTIAL_DOUBLES);
    if (chunks_out) *chunks_out = chunks;
    const size_t part_doubles = (size_t)g * nblocks * nv + (size_t)g;  // rows, then counts
    return sizeof(double) * (part_doubles + diag_partial_doubles(m, per_launch, grad, chunks)) + 256;
}

// Scratch of an FP32 grid call (grid workspace, then per-setting counts).
size_t grid_call_scratch(const cde_model* m, int n_hx, int n_hy)
{
    return grid_work_bytes(m, n_hx, n_hy) + sizeof(double) * (size_t)n_hx * n_hy + 256;
}

// The pass itself, in `work` (block rows and counts, then the chunk partials
// of `chunks` j-chunks per launch: diag_list_scratch's layout).
template <typename T>
cde_status run_diag_list_in(const cde_model* m, const double* h, int g, int crit, bool grad,
                            double* totals, double* grad_out, double* per_point, int64_t* nonfinite,
                            int chunks, void* work, hipStream_t stream)
{
    const int p = m->dx + m->dy;
    const int nblocks = (int)(m->npad / TILE);
    const int nv = grad ? p + 2 : 2;
    const size_t part_doubles = (size_t)g * nblocks * nv + (size_t)g;
    double* part = (double*)work;
    double* partial = part + part_doubles;
    for (int s0 = 0; s0 < g; s0 += MAX_SETS_PER_LAUNCH) {
        const int cnt = std::min(MAX_SETS_PER_LAUNCH, g - s0);
        DiagSets<T> sets;
        std::memset(&sets, 0, sizeof sets);
        for (int s = 0; s < cnt; ++s) fill_set(sets.s[s], h + (size_t)(s0 + s) * p, m->dx, m->dy);
        hipError_t e = launch_diag<T>(m, sets, cnt, crit, grad, chunks, partial,
                                      per_point ? per_point + (size_t)s0 * m->n : nullptr,
                                      part + (size_t)s0 * nblocks * nv, stream);
        if (e != hipSuccess) return hip_fail(e, "launch k_loo_diag");
    }
    double* counts = part + (size_t)g * nblocks * nv;
    hipError_t e = launch_reduce_parts(part, g, nblocks, nv, totals, grad ? grad_out : nullptr,
                                       counts, nonfinite, stream);
    if (e != hipSuccess) return hip_fail(e, "launch k_reduce_parts");
    return CDE_OK;
}

template <typename T>
cde_status run_diag_list(cde_model* m, const double* h, int g, int crit, bool grad, double* totals,
                         double* grad_out, double* per_point, int64_t* nonfinite,
                         hipStream_t stream)
{
    int chunks = 1;
    const size_t scratch = diag_list_scratch<T>(m, g, grad, &chunks);
    cde_status st = ensure_scratch(m, scratch);
    if (st != CDE_OK) return st;
    return run_diag_list_in<T>(m, h, g, crit, grad, totals, grad_out, per_point, nonfinite, chunks,
                               m->scratch, stream);
}

// ---- the allocation-free value and gradient (cde_loo_grad_noalloc) ----
//
// Its scratch is this file-scope device array: one copy per GPU, created when
// the library's code is loaded on that GPU and held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): the device address of each GPU's copy is
// read once with hipGetSymbolAddress, with that GPU current, and kept in
// g_noalloc_ptr.  Every call on a GPU shares its copy, so calls that overlap
// in time on one GPU race.  The pass writes every scratch value it reads, so
// nothing needs clearing between calls.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current GPU's copy of noalloc_scratch.
cde_status noalloc_scratch_ptr(int device, void** out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return fail(CDE_EUNSUPPORTED, "cde_loo_grad_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(noalloc_scratch)");
        g_noalloc_ptr[device] = p;
    }
    *out = g_noalloc_ptr[device];
    return CDE_OK;
}

// Value and gradient of one setting with the scratch above: the j-chunk count
// of cde_loo_grad, reduced until the chunk partials fit.
template <typename T>
cde_status run_grad_noalloc(cde_model* m, const double* h, int crit, double* total, double* grad,
                            double* per_point, hipStream_t stream)
{
    const int nblocks = (int)(m->npad / TILE);
    const int nv = m->dx + m->dy + 2;
    const size_t rows_bytes = sizeof(double) * ((size_t)nblocks * nv + 1);
    if (rows_bytes + 256 >= NOALLOC_SCRATCH_BYTES)
        return fail(CDE_EUNSUPPORTED, "cde_loo_grad_noalloc: n too large for the 64 MiB scratch");
    const size_t max_doubles = (NOALLOC_SCRATCH_BYTES - rows_bytes - 256) / sizeof(double);
    if (diag_partial_doubles(m, 1, true, 1) > max_doubles) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "cde_loo_grad_noalloc: n = %lld needs %zu bytes of scratch, more than the "
                      "64 MiB the entry point holds",
                      (long long)m->n, rows_bytes + sizeof(double) * diag_partial_doubles(m, 1, true, 1));
        return fail(CDE_EUNSUPPORTED, msg);
    }
    const int chunks = diag_chunks<T>(m, 1, true, std::min(max_doubles, MAX_DIAG_PARTIAL_DOUBLES));
    void* work = nullptr;
    cde_status st = noalloc_scratch_ptr(m->device, &work);
    if (st != CDE_OK) return st;
    return run_diag_list_in<T>(m, h, 1, crit, true, total, grad, per_point, nullptr, chunks, work, stream);
}

void fill_epan(EpanSet& s, const double* h, int dx, int dy)
{
    std::memset(&s, 0, sizeof s);
    for (int k = 0; k < dx + dy; ++k) s.inv_h[k] = 1.0 / h[k];
    s.log_cx = log_epan_norm(h, dx);
    s.log_cy = log_epan_norm(h + dx, dy);
}

// Spatial order of the points, built on first use (one-time device memory:
// sorted FP64 rows, permutation, tile boxes).
cde_status ensure_index(cde_model* m, hipStream_t stream)
{
    if (m->index_ready) return CDE_OK;
    const size_t spts_bytes = sizeof(double) * (size_t)m->npad * m->stride;
    const size_t perm_bytes = sizeof(int) * (size_t)m->npad;
    const size_t box_bytes = sizeof(double) * (size_t)(m->npad / TILE) * 2 * m->dx;
    const size_t sbox_bytes = sizeof(double) * (size_t)(m->npad / SUBROWS) * 2 * m->dx;
    struct {
        void** p;
        size_t b;
        const char* what;
    } allocs[] = {{&m->spts, spts_bytes, "hipMalloc(sorted points)"},
                  {&m->perm, perm_bytes, "hipMalloc(permutation)"},
                  {&m->tbox, box_bytes, "hipMalloc(tile boxes)"},
                  {&m->sbox, sbox_bytes, "hipMalloc(subtile boxes)"}};
    for (auto& a : allocs) {
        if (*a.p) continue;
        hipError_t e = hipMalloc(a.p, a.b);
        if (e != hipSuccess) {
            *a.p = nullptr;
            return hip_fail(e, a.what);
        }
        m->bytes += a.b;
    }
    const size_t wb = index_work_bytes(m);
    cde_status st = ensure_scratch(m, wb);
    if (st != CDE_OK) return st;
    hipError_t e = launch_build_index(m, m->scratch, m->scratch_bytes, stream);
    if (e != hipSuccess) return hip_fail(e, "build spatial index");
    m->index_ready = true;
    return CDE_OK;
}

// Epanechnikov values for a list of g diagonal settings: totals[g], per-point
// values in the caller's order, per-setting non-finite counts summed into
// *nonfinite when given.
cde_status run_epan_list(cde_model* m, const double* h, int g, int crit, double* totals,
                         double* per_point, int64_t* nonfinite, hipStream_t stream)
{
    cde_status st = ensure_index(m, stream);
    if (st != CDE_OK) return st;
    const int p = m->dx + m->dy;
    const int nblocks = (int)(m->npad / TILE);
    const int per_launch = std::min(g, MAX_SETS_PER_LAUNCH);
    const int chunks = epan_chunks(m, per_launch, MAX_DIAG_PARTIAL_DOUBLES);
    const size_t part_doubles = (size_t)g * nblocks * 2 + (size_t)g;
    const size_t partial_doubles = (size_t)per_launch * chunks * 2 * (size_t)m->npad;
    st = ensure_scratch(m, sizeof(double) * (part_doubles + partial_doubles) + 256);
    if (st != CDE_OK) return st;
    double* part = (double*)m->scratch;
    double* partial = part + part_doubles;
    for (int s0 = 0; s0 < g; s0 += MAX_SETS_PER_LAUNCH) {
        const int cnt = std::min(MAX_SETS_PER_LAUNCH, g - s0);
        EpanSets sets;
        std::memset(&sets, 0, sizeof sets);
        for (int s = 0; s < cnt; ++s) fill_epan(sets.s[s], h + (size_t)(s0 + s) * p, m->dx, m->dy);
        hipError_t e = launch_epan(m, sets, cnt, crit, chunks, partial,
                                   per_point ? per_point + (size_t)s0 * m->n : nullptr,
                                   part + (size_t)s0 * nblocks * 2, stream);
        if (e != hipSuccess) return hip_fail(e, "launch k_loo_epan");
    }
    double* counts = part + (size_t)g * nblocks * 2;
    hipError_t e = launch_reduce_parts(part, g, nblocks, 2, totals, nullptr, counts, nonfinite, stream);
    if (e != hipSuccess) return hip_fail(e, "launch k_reduce_parts");
    return CDE_OK;
}

}  // namespace

extern "C" {

int cde_abi_version(void) { return CDE_ABI_VERSION; }

const char* cde_last_error(void) { return g_last_error.c_str(); }

cde_status cde_create(cde_model** out, const void* x_dev, const void* y_dev, int64_t n, int32_t dx,
                      int32_t dy, cde_precision precision, void* stream)
{
    try {
        if (!out) return fail(CDE_EINVAL, "cde_create: out is NULL");
        *out = nullptr;
        if (!x_dev || !y_dev) return fail(CDE_EINVAL, "cde_create: x_dev or y_dev is NULL");
        if (n < 2) return fail(CDE_EINVAL, "cde_create: n must be >= 2");
        if (n >= (int64_t(1) << 31) - TILE) return fail(CDE_EUNSUPPORTED, "cde_create: n >= 2^31");
        if (dx < 1 || dy < 1) return fail(CDE_EINVAL, "cde_create: dx and dy must be >= 1");
        if (!supported_dims(dx, dy))
            return fail(CDE_EUNSUPPORTED, "cde_create: supported shapes are dx in {1..8, 16}, dy in {1, 2}");
        if (precision != CDE_F32 && precision != CDE_F64)
            return fail(CDE_EINVAL, "cde_create: unknown precision");
        cde_model* m = new (std::nothrow) cde_model;
        if (!m) return fail(CDE_ENOMEM, "cde_create: host allocation failed");
        m->n = n;
        m->npad = (n + TILE - 1) / TILE * TILE;
        m->dx = dx;
        m->dy = dy;
        m->stride = row_stride(dx, dy);
        m->prec = precision;
        hipError_t e = hipGetDevice(&m->device);
        if (e != hipSuccess) { delete m; return hip_fail(e, "hipGetDevice"); }
        e = hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, m->device);
        if (e != hipSuccess) { delete m; return hip_fail(e, "hipDeviceGetAttribute"); }
        const size_t elt = precision == CDE_F64 ? sizeof(double) : sizeof(float);
        const size_t pts_bytes = packed_bytes(m->npad, m->stride, elt);
        e = hipMalloc(&m->pts, pts_bytes);
        if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(points)"); }
        m->bytes = pts_bytes;
        m->ext_dev = (unsigned long long*)((char*)m->pts + (pts_bytes - EXT_BYTES));
        auto undo = [&](hipError_t err, const char* what) {
            if (m->ext_event) (void)hipEventDestroy(m->ext_event);
            if (m->ext_host) (void)hipHostFree(m->ext_host);
            (void)hipFree(m->pts);
            delete m;
            return hip_fail(err, what);
        };
        e = hipHostMalloc((void**)&m->ext_host, EXT_BYTES, hipHostMallocDefault);
        if (e != hipSuccess) { m->ext_host = nullptr; return undo(e, "hipHostMalloc(data extent)"); }
        e = hipEventCreateWithFlags(&m->ext_event, hipEventDisableTiming);
        if (e != hipSuccess) { m->ext_event = nullptr; return undo(e, "hipEventCreate"); }
        hipStream_t s = (hipStream_t)stream;
        e = precision == CDE_F64 ? launch_pack<double>(m, (const double*)x_dev, (const double*)y_dev, s)
                                 : launch_pack<float>(m, (const float*)x_dev, (const float*)y_dev, s);
        if (e != hipSuccess) return undo(e, "launch k_pack");
        e = precision == CDE_F64 ? launch_extent<double>(m, m->ext_dev, s) : launch_extent<float>(m, m->ext_dev, s);
        if (e != hipSuccess) return undo(e, "launch k_extent");
        e = hipMemcpyAsync(m->ext_host, m->ext_dev, sizeof(unsigned long long) * (2 * MAXP + 1),
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return undo(e, "hipMemcpyAsync(data extent)");
        e = hipEventRecord(m->ext_event, s);
        if (e != hipSuccess) return undo(e, "hipEventRecord(data extent)");
        *out = m;
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_create: unexpected exception");
    }
}

cde_status cde_destroy(cde_model* m)
{
    if (!m) return CDE_OK;
    DeviceGuard guard(m->device);
    cde_status st = CDE_OK;
    if (m->ext_event) {
        hipError_t e = hipEventSynchronize(m->ext_event);  // the extent copy targets ext_host
        if (e == hipSuccess) e = hipEventDestroy(m->ext_event);
        if (e != hipSuccess && st == CDE_OK) st = hip_fail(e, "hipEventDestroy");
    }
    if (m->ext_host) {
        hipError_t e = hipHostFree(m->ext_host);
        if (e != hipSuccess && st == CDE_OK) st = hip_fail(e, "hipHostFree");
    }
    for (void* p : {m->pts, m->nn, m->xmean, m->spts, m->perm, m->tbox, m->sbox, m->scratch}) {
        if (!p) continue;
        hipError_t e = hipFree(p);
        if (e != hipSuccess && st == CDE_OK) st = hip_fail(e, "hipFree");
    }
    delete m;
    return st;
}

size_t cde_model_device_bytes(const cde_model* m) { return m ? m->bytes : 0; }

size_t cde_workspace_bytes(int64_t n, int32_t dx, int32_t dy, cde_precision precision, int32_t n_hx,
                           int32_t n_hy)
{
    try {
        if (n < 2 || n >= (int64_t(1) << 31) - TILE || !supported_dims(dx, dy)) return 0;
        if (precision != CDE_F32 && precision != CDE_F64) return 0;
        if (n_hx < 0 || n_hy < 0 || n_hx > 64 || n_hy > 64 || (n_hx == 0) != (n_hy == 0)) return 0;
        cde_model t;  // shape only: no device memory
        t.n = n;
        t.npad = (n + TILE - 1) / TILE * TILE;
        t.dx = dx;
        t.dy = dy;
        t.stride = row_stride(dx, dy);
        t.prec = precision;
        if (hipGetDevice(&t.device) != hipSuccess ||
            hipDeviceGetAttribute(&t.ncu, hipDeviceAttributeMultiprocessorCount, t.device) != hipSuccess)
            t.ncu = 0;
        const size_t elt = precision == CDE_F64 ? sizeof(double) : sizeof(float);
        size_t bytes = packed_bytes(t.npad, t.stride, elt);
        if (n_hx == 0) return bytes;
        if (precision == CDE_F64)
            return bytes + round_scratch(diag_list_scratch<double>(&t, n_hx * n_hy, false, nullptr));
        return bytes + sizeof(double) * 2 * (size_t)t.npad +
               round_scratch(grid_call_scratch(&t, n_hx, n_hy));
    } catch (...) {
        return 0;
    }
}

cde_status cde_check_bandwidths(const double* range, int32_t dx, int32_t dy, const double* h,
                                cde_precision precision, int32_t diagonal_pass)
{
    try {
        if (!range || !h) return fail(CDE_EINVAL, "cde_check_bandwidths: NULL pointer");
        if (dx < 1 || dy < 1 || dx + dy > MAXP)
            return fail(CDE_EINVAL, "cde_check_bandwidths: need dx, dy >= 1 and dx + dy <= 18");
        if (precision != CDE_F32 && precision != CDE_F64)
            return fail(CDE_EINVAL, "cde_check_bandwidths: unknown precision");
        for (int k = 0; k < dx + dy; ++k)
            if (!(range[k] >= 0.0) || !std::isfinite(range[k]))
                return fail(CDE_EINVAL, "cde_check_bandwidths: ranges must be finite and >= 0");
        if (!valid_bandwidths(h, dx + dy))
            return fail(CDE_EINVAL, "cde_check_bandwidths: bandwidths must be finite and > 0");
        return check_setting(range, dx, dy, h, precision, diagonal_pass != 0, "cde_check_bandwidths");
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_check_bandwidths: unexpected exception");
    }
}

cde_status cde_loo_loglik_list(cde_model* m, const double* h, int32_t g, cde_criterion criterion,
                               cde_kernel kernel, double* totals_dev, double* per_point_dev,
                               void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_loo_loglik_list: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_loo_loglik_list"); st0 != CDE_OK) return st0;
        if (!totals_dev) return fail(CDE_EINVAL, "cde_loo_loglik_list: totals_dev is NULL");
        if (g < 1 || g > 4096) return fail(CDE_EINVAL, "cde_loo_loglik_list: g must be in [1, 4096]");
        if (criterion != CDE_COND && criterion != CDE_JOINT)
            return fail(CDE_EINVAL, "cde_loo_loglik_list: unknown criterion");
        if (kernel != CDE_GAUSSIAN && kernel != CDE_EPANECHNIKOV)
            return fail(CDE_EINVAL, "cde_loo_loglik_list: unknown kernel");
        cde_status st = check_model_settings(m, h, g, kernel == CDE_GAUSSIAN, "cde_loo_loglik_list");
        if (st != CDE_OK) return st;
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        if (kernel == CDE_EPANECHNIKOV)
            return run_epan_list(m, h, g, criterion, totals_dev, per_point_dev, nullptr, s);
        return m->prec == CDE_F64
                   ? run_diag_list<double>(m, h, g, criterion, false, totals_dev, nullptr,
                                           per_point_dev, nullptr, s)
                   : run_diag_list<float>(m, h, g, criterion, false, totals_dev, nullptr,
                                          per_point_dev, nullptr, s);
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_loo_loglik_list: unexpected exception");
    }
}

cde_status cde_loo_loglik(cde_model* m, const double* hx, int32_t n_hx, const double* hy,
                          int32_t n_hy, cde_criterion criterion, cde_kernel kernel, cde_xterm xterm,
                          double* totals_dev, double* per_point_dev, int64_t* n_nonfinite_dev,
                          void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_loo_loglik: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_loo_loglik"); st0 != CDE_OK) return st0;
        if (!totals_dev) return fail(CDE_EINVAL, "cde_loo_loglik: totals_dev is NULL");
        if (n_hx < 1 || n_hx > 64 || n_hy < 1 || n_hy > 64)
            return fail(CDE_EINVAL, "cde_loo_loglik: grid sizes must be in [1, 64]");
        if (criterion != CDE_COND && criterion != CDE_JOINT)
            return fail(CDE_EINVAL, "cde_loo_loglik: unknown criterion");
        if (xterm != CDE_XTERM_AUTO && xterm != CDE_XTERM_VALU && xterm != CDE_XTERM_MFMA_BF16X3 &&
            xterm != CDE_XTERM_VALU_F32)
            return fail(CDE_EINVAL, "cde_loo_loglik: unknown xterm");
        if (kernel != CDE_GAUSSIAN && kernel != CDE_EPANECHNIKOV)
            return fail(CDE_EINVAL, "cde_loo_loglik: unknown kernel");
        // distance variant of the FP32 grid pass: 0 FP64 differences, 1 FP32
        // differences, 2 split-bf16 x3 cross term
        const int xm = xterm == CDE_XTERM_MFMA_BF16X3 ? 2 : xterm == CDE_XTERM_VALU_F32 ? 1 : 0;
        const bool xt = xm == 2;
        if (xm != 0 && (m->dx != 16 || m->prec != CDE_F32 || kernel != CDE_GAUSSIAN))
            return fail(CDE_EUNSUPPORTED,
                        "cde_loo_loglik: the FP32-difference and MFMA cross-term options need dx = 16, FP32 "
                        "data and the Gaussian kernel");
        {
            cde_status st = check_model_grid(m, hx, n_hx, hy, n_hy, m->prec == CDE_F64 && kernel == CDE_GAUSSIAN,
                                             "cde_loo_loglik");
            if (st != CDE_OK) return st;
        }
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        const int g = n_hx * n_hy;
        if (m->prec == CDE_F64 || kernel == CDE_EPANECHNIKOV) {
            // FP64 models, and the Epanechnikov kernel: every setting as a
            // diagonal setting (FP64 throughout).
            const int p = m->dx + m->dy;
            std::vector<double> h((size_t)g * p);
            for (int a = 0; a < n_hx; ++a)
                for (int b = 0; b < n_hy; ++b)
                    for (int k = 0; k < p; ++k)
                        h[(size_t)(a * n_hy + b) * p + k] = k < m->dx ? hx[a] : hy[b];
            if (kernel == CDE_EPANECHNIKOV)
                return run_epan_list(m, h.data(), g, criterion, totals_dev, per_point_dev,
                                     n_nonfinite_dev, s);
            return run_diag_list<double>(m, h.data(), g, criterion, false, totals_dev, nullptr,
                                         per_point_dev, n_nonfinite_dev, s);
        }
        if (!m->nn) {
            hipError_t e = hipMalloc(&m->nn, sizeof(double) * 2 * (size_t)m->npad);
            if (e != hipSuccess) {
                m->nn = nullptr;
                return hip_fail(e, "hipMalloc(neighbour shifts)");
            }
            m->bytes += sizeof(double) * 2 * (size_t)m->npad;
        }
        if (xt && !m->xmean) {
            hipError_t e = hipMalloc(&m->xmean, 16 * sizeof(float));
            if (e != hipSuccess) {
                m->xmean = nullptr;
                return hip_fail(e, "hipMalloc(column means)");
            }
            m->bytes += 16 * sizeof(float);
        }
        const size_t wb = grid_work_bytes(m, n_hx, n_hy);
        cde_status st = ensure_scratch(m, grid_call_scratch(m, n_hx, n_hy));
        if (st != CDE_OK) return st;
        double* counts = (double*)((char*)m->scratch + wb);
        hipError_t e = launch_grid(m, hx, n_hx, hy, n_hy, criterion, xm, totals_dev, per_point_dev,
                                   m->scratch, wb, counts, s);
        if (e != hipSuccess) return hip_fail(e, "launch grid kernels");
        m->nn_ready = true;
        if (n_nonfinite_dev) {
            e = launch_sum_counts(counts, g, n_nonfinite_dev, s);
            if (e != hipSuccess) return hip_fail(e, "launch k_sum_counts");
        }
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_loo_loglik: unexpected exception");
    }
}

cde_status cde_loo_grad(cde_model* m, const double* h, cde_criterion criterion, double* total_dev,
                        double* grad_dev, double* per_point_dev, void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_loo_grad: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_loo_grad"); st0 != CDE_OK) return st0;
        if (!total_dev || !grad_dev) return fail(CDE_EINVAL, "cde_loo_grad: output pointer is NULL");
        if (criterion != CDE_COND && criterion != CDE_JOINT)
            return fail(CDE_EINVAL, "cde_loo_grad: unknown criterion");
        {
            cde_status st = check_model_settings(m, h, 1, true, "cde_loo_grad");
            if (st != CDE_OK) return st;
        }
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        return m->prec == CDE_F64
                   ? run_diag_list<double>(m, h, 1, criterion, true, total_dev, grad_dev,
                                           per_point_dev, nullptr, s)
                   : run_diag_list<float>(m, h, 1, criterion, true, total_dev, grad_dev,
                                          per_point_dev, nullptr, s);
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_loo_grad: unexpected exception");
    }
}

cde_status cde_launch_batch(const cde_work_item* items, int32_t n_items, const double* hx, int32_t n_hx,
                            const double* hy, int32_t n_hy, cde_criterion criterion, void* stream)
{
    try {
        if (!items || n_items < 1 || n_items > 512)
            return fail(CDE_EINVAL, "cde_launch_batch: need 1 <= n_items <= 512 and items != NULL");
        if (!hx || !hy) return fail(CDE_EINVAL, "cde_launch_batch: hx or hy is NULL");
        if (n_hx < 1 || n_hx > 16 || n_hy < 1 || n_hy > 16)
            return fail(CDE_EINVAL, "cde_launch_batch: grid sizes must be in [1, 16]");
        if (criterion != CDE_COND && criterion != CDE_JOINT)
            return fail(CDE_EINVAL, "cde_launch_batch: unknown criterion");
        const cde_model* m0 = items[0].model;
        if (!m0) return fail(CDE_EINVAL, "cde_launch_batch: item 0 has no model");
        const uint64_t sig = grid_signature(hx, n_hx, hy, n_hy, criterion);
        std::vector<GridRange> ranges((size_t)n_items);
        for (int k = 0; k < n_items; ++k) {
            const cde_work_item& it = items[k];
            cde_model* m = it.model;
            char who[64];
            std::snprintf(who, sizeof who, "cde_launch_batch: item %d", k);
            if (!m) return fail(CDE_EINVAL, std::string(who) + " has no model");
            if (m->prec != CDE_F32) return fail(CDE_EUNSUPPORTED, std::string(who) + ": FP32 models only");
            if (m->dx != m0->dx || m->dy != m0->dy || m->device != m0->device)
                return fail(CDE_EINVAL, std::string(who) + ": items must share dx, dy and the device");
            for (int q = 0; q < k; ++q)
                if (items[q].model == m) return fail(CDE_EINVAL, std::string(who) + ": model listed twice");
            if (!(it.i0 >= 0 && it.i0 < it.i1 && it.i1 <= m->n) || it.i0 % TILE != 0 ||
                (it.i1 != m->n && it.i1 % TILE != 0))
                return fail(CDE_EINVAL, std::string(who) +
                                            ": need 0 <= i0 < i1 <= n, i0 a multiple of 256 and i1 one "
                                            "or n");
            if (it.i1 == m->n && !it.totals_dev)
                return fail(CDE_EINVAL, std::string(who) + ": the range ending at n needs totals_dev");
            if (it.i0 != m->batch_next)
                return fail(CDE_EINVAL, std::string(who) + ": ranges of a model must follow each other "
                                                           "from 0 (expected i0 = " +
                                            std::to_string((long long)m->batch_next) + ")");
            if (it.i0 > 0 && sig != m->batch_sig)
                return fail(CDE_EINVAL, std::string(who) + ": grid or criterion changed within an evaluation");
            cde_status st = check_model_grid(m, hx, n_hx, hy, n_hy, false, who);
            if (st != CDE_OK) return st;
        }
        DeviceGuard guard(m0->device);
        if (!guard.ok) return fail(CDE_EDEVICE, "cde_launch_batch: cannot make the models' device current");
        for (int k = 0; k < n_items; ++k) {
            cde_model* m = items[k].model;
            const size_t wb = grid_work_bytes(m, n_hx, n_hy);
            const size_t need = grid_call_scratch(m, n_hx, n_hy);
            if (items[k].i0 == 0) {
                if (!m->nn) {
                    hipError_t e = hipMalloc(&m->nn, sizeof(double) * 2 * (size_t)m->npad);
                    if (e != hipSuccess) {
                        m->nn = nullptr;
                        return hip_fail(e, "hipMalloc(neighbour shifts)");
                    }
                    m->bytes += sizeof(double) * 2 * (size_t)m->npad;
                }
                cde_status st = ensure_scratch(m, need);
                if (st != CDE_OK) return st;
            } else if (m->scratch_bytes < need) {
                return fail(CDE_EINVAL, "cde_launch_batch: model scratch shrank within an evaluation");
            }
            GridRange& r = ranges[k];
            r.m = m;
            r.i0 = items[k].i0;
            r.i1 = items[k].i1;
            r.totals = items[k].totals_dev;
            r.nonfinite = items[k].n_nonfinite_dev;
            r.work = m->scratch;
            r.work_bytes = wb;
            r.counts = (double*)((char*)m->scratch + wb);
            r.do_nn = !m->nn_ready;
        }
        hipError_t e = launch_grid_batch(ranges.data(), n_items, hx, n_hx, hy, n_hy, criterion,
                                         (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "launch grouped grid kernels");
        for (int k = 0; k < n_items; ++k) {
            cde_model* m = items[k].model;
            const bool last = items[k].i1 == m->n;
            m->batch_next = last ? 0 : items[k].i1;
            m->batch_sig = sig;
            if (last) m->nn_ready = true;
        }
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_launch_batch: unexpected exception");
    }
}

int64_t cde_batch_round_points(int32_t dx, int32_t dy)
{
    try {
        if (!supported_dims(dx, dy)) return 0;
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        return grid_round_points(dx, dy, ncu);
    } catch (...) {
        return 0;
    }
}

cde_status cde_loo_grad_noalloc(cde_model* m, const double* h, cde_criterion criterion,
                                double* total_dev, double* grad_dev, double* per_point_dev,
                                void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_loo_grad_noalloc: model is NULL");
        if (!total_dev || !grad_dev) return fail(CDE_EINVAL, "cde_loo_grad_noalloc: output pointer is NULL");
        if (criterion != CDE_COND && criterion != CDE_JOINT)
            return fail(CDE_EINVAL, "cde_loo_grad_noalloc: unknown criterion");
        {
            cde_status st = check_model_settings(m, h, 1, true, "cde_loo_grad_noalloc");
            if (st != CDE_OK) return st;
        }
        DeviceGuard guard(m->device);
        if (!guard.ok) return fail(CDE_EDEVICE, "cde_loo_grad_noalloc: cannot make the model's device current");
        hipStream_t s = (hipStream_t)stream;
        return m->prec == CDE_F64
                   ? run_grad_noalloc<double>(m, h, criterion, total_dev, grad_dev, per_point_dev, s)
                   : run_grad_noalloc<float>(m, h, criterion, total_dev, grad_dev, per_point_dev, s);
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_loo_grad_noalloc: unexpected exception");
    }
}

cde_status cde_cv_ise(cde_model* m, const double* h, double* out_dev, double* terms_dev, void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_cv_ise: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_cv_ise"); st0 != CDE_OK) return st0;
        if (!out_dev) return fail(CDE_EINVAL, "cde_cv_ise: output pointer is NULL");
        if (m->prec != CDE_F32) return fail(CDE_EUNSUPPORTED, "cde_cv_ise: FP32 models only");
        {
            cde_status st = check_model_settings(m, h, 1, true, "cde_cv_ise");
            if (st != CDE_OK) return st;
        }
        if (m->n > CDE_ISE_MAX_N) return fail(CDE_EUNSUPPORTED, "cde_cv_ise: n > 262144");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = m->n;
        // scratch: the LOO pass's own scratch, then l_i [n], the LOO total,
        // the terms (unless the caller takes them) and the ISE work area
        const size_t diag = round_scratch(diag_list_scratch<float>(m, 1, false, nullptr));
        const size_t extra = sizeof(double) * ((size_t)n + 8 + (terms_dev ? 0 : 2 * (size_t)n) +
                                               ise_work_doubles(m)) + 256;
        cde_status st = ensure_scratch(m, diag + extra);
        if (st != CDE_OK) return st;
        double* ell = (double*)((char*)m->scratch + diag);
        double* loo_total = ell + n;
        double* terms = terms_dev ? terms_dev : loo_total + 8;
        double* work = terms_dev ? loo_total + 8 : terms + 2 * n;
        st = run_diag_list<float>(m, h, 1, CDE_COND, false, loo_total, nullptr, ell, nullptr, s);
        if (st != CDE_OK) return st;
        hipError_t e = launch_cv_ise(m, h, ell, out_dev, terms, work, s);
        if (e != hipSuccess) return hip_fail(e, "launch k_ise");
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_cv_ise: unexpected exception");
    }
}

cde_status cde_density_query(cde_model* m, const void* xq_dev, int64_t q, const void* ygrid_dev,
                             int64_t k, const double* h, cde_kernel kernel, double* f_dev, void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_density_query: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_density_query"); st0 != CDE_OK) return st0;
        if (kernel != CDE_GAUSSIAN && kernel != CDE_EPANECHNIKOV)
            return fail(CDE_EINVAL, "cde_density_query: unknown kernel");
        if (q < 0 || k < 0 || k > 4096) return fail(CDE_EINVAL, "cde_density_query: need q >= 0, 0 <= k <= 4096");
        if (q > 0 && k > 0 && (!xq_dev || !ygrid_dev || !f_dev))
            return fail(CDE_EINVAL, "cde_density_query: NULL device pointer");
        {
            cde_status st = check_model_settings(m, h, 1, m->prec == CDE_F64 && kernel == CDE_GAUSSIAN,
                                                 "cde_density_query");
            if (st != CDE_OK) return st;
        }
        if (q == 0 || k == 0) return CDE_OK;
        if (q * k >= (int64_t(1) << 40)) return fail(CDE_EUNSUPPORTED, "cde_density_query: q*k too large");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        hipError_t e;
        if (m->prec == CDE_F64) {
            if (kernel != CDE_GAUSSIAN)
                return fail(CDE_EUNSUPPORTED, "cde_density_query: Epanechnikov queries need an FP32 model");
            DiagSets<double> sets;
            std::memset(&sets, 0, sizeof sets);
            fill_set(sets.s[0], h, m->dx, m->dy);
            e = launch_query<double>(m, (const double*)xq_dev, q, (const double*)ygrid_dev, k, sets,
                                     f_dev, s);
        } else {
            if (q >= (int64_t(1) << 31) - 64) return fail(CDE_EUNSUPPORTED, "cde_density_query: q >= 2^31");
            if (kernel == CDE_EPANECHNIKOV) {
                cde_status st = ensure_index(m, s);
                if (st != CDE_OK) return st;
                st = ensure_scratch(m, query_epan_work_bytes(m, q, k) + 256);
                if (st != CDE_OK) return st;
                e = launch_query_epan(m, (const float*)xq_dev, (int)q, (const float*)ygrid_dev, (int)k, h,
                                      f_dev, (char*)m->scratch, s);
            } else {
                cde_status st = ensure_scratch(m, sizeof(double) * query_work_doubles(m, q, k) + 256);
                if (st != CDE_OK) return st;
                e = launch_query_mfma(m, (const float*)xq_dev, (int)q, (const float*)ygrid_dev, (int)k, h,
                                      f_dev, (double*)m->scratch, s);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "launch k_query");
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_density_query: unexpected exception");
    }
}

cde_status cde_conditional_mean(cde_model* m, const void* xq_dev, int64_t q, const double* h,
                                double* mean_dev, void* stream)
{
    try {
        if (!m) return fail(CDE_EINVAL, "cde_conditional_mean: model is NULL");
        if (cde_status st0 = reject_if_batching(m, "cde_conditional_mean"); st0 != CDE_OK) return st0;
        if (q < 0) return fail(CDE_EINVAL, "cde_conditional_mean: q must be >= 0");
        if (q > 0 && (!xq_dev || !mean_dev)) return fail(CDE_EINVAL, "cde_conditional_mean: NULL device pointer");
        {
            cde_status st = check_model_settings(m, h, 1, false, "cde_conditional_mean");
            if (st != CDE_OK) return st;
        }
        if (q == 0) return CDE_OK;
        if (q >= (int64_t(1) << 40)) return fail(CDE_EUNSUPPORTED, "cde_conditional_mean: q too large");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        cde_status st = ensure_scratch(m, sizeof(double) * cond_mean_work_doubles(m, q) + 256);
        if (st != CDE_OK) return st;
        hipError_t e = launch_cond_mean(m, xq_dev, q, h, mean_dev, (double*)m->scratch, s);
        if (e != hipSuccess) return hip_fail(e, "launch conditional mean");
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_conditional_mean: unexpected exception");
    }
}

cde_status cde_density_summary(const double* f_dev, const double* ygrid_dev, int64_t q, int64_t k,
                               double alpha, double* out_dev, void* stream)
{
    try {
        if (q < 0 || k < 2 || k > 4096) return fail(CDE_EINVAL, "cde_density_summary: need q >= 0, 2 <= k <= 4096");
        if (!(alpha > 0.0) || !(alpha < 1.0)) return fail(CDE_EINVAL, "cde_density_summary: alpha must be in (0, 1)");
        if (q > 0 && (!f_dev || !ygrid_dev || !out_dev))
            return fail(CDE_EINVAL, "cde_density_summary: NULL device pointer");
        if (q == 0) return CDE_OK;
        if (q >= (int64_t(1) << 31)) return fail(CDE_EUNSUPPORTED, "cde_density_summary: q >= 2^31");
        hipError_t e = launch_density_summary(f_dev, ygrid_dev, q, k, alpha, out_dev, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "launch density summary");
        return CDE_OK;
    } catch (...) {
        return fail(CDE_EDEVICE, "cde_density_summary: unexpected exception");
    }
}

}  // extern "C"
