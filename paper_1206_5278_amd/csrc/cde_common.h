// cde_common.h -- definitions shared by the host API and the gfx950 kernels of
// the exact LOO likelihood library (see include/cde.h for the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cde.h"

namespace cde {

constexpr int TILE = 256;           // points per tile (i-block and j-tile)
constexpr int SUBROWS = 32;         // rows per subtile box of the spatial index
constexpr int MAXP = 18;            // dx + dy for the largest instantiated shape (16 + 2)
constexpr double LOG2E = 1.4426950408889634073599246810019;
constexpr double LN2 = 0.69314718055994530941723212145818;
constexpr double HALF_LOG_2PI = 0.91893853320467274178032973640562;
constexpr int64_t CDE_ISE_MAX_N = 262144;  // largest n of the cross-validated ISE

// Points are stored array-of-structures, x then y then zero padding, with a
// row stride rounded up to 4 values so that a whole point is one or more
// 16-byte (FP32) loads.
__host__ __device__ constexpr int row_stride(int dx, int dy) { return ((dx + dy + 3) / 4) * 4; }

// One diagonal bandwidth setting, as the kernels consume it.  c[k] is the
// Gaussian exponent coefficient in base 2, log2(e) / (2 h_k^2), so that a
// kernel value is exp2(-sum_k c_k d_k^2) times its normalising constant.
template <typename T>
struct DiagSet {
    T c[MAXP];
    double inv_h[MAXP];    // 1 / h_k
    double inv_h3[MAXP];   // 1 / h_k^3
    double log_cx;         // -sum_k (log hx_k + log(2 pi)/2)
    double log_cy;         // -sum_l (log hy_l + log(2 pi)/2)
};

constexpr int MAX_SETS_PER_LAUNCH = 8;
// One diagonal setting for the Epanechnikov kernel: inverse bandwidths and
// the log normalisations log c_x, log c_y of the radial kernel.
struct EpanSet {
    double inv_h[MAXP];
    double log_cx;
    double log_cy;
};
struct EpanSets {
    EpanSet s[MAX_SETS_PER_LAUNCH];
};

// Cap on the chunk partials of one diagonal launch (2 GiB of doubles).
constexpr size_t MAX_DIAG_PARTIAL_DOUBLES = size_t(1) << 28;

template <typename T>
struct DiagSets {
    DiagSet<T> s[MAX_SETS_PER_LAUNCH];
};

}  // namespace cde

// The opaque model handle of the C ABI.
struct cde_model {
    int64_t n = 0;
    int64_t npad = 0;        // n rounded up to a whole number of tiles
    int32_t dx = 0, dy = 0, stride = 0;
    cde_precision prec = CDE_F32;
    int device = 0;
    int ncu = 0;             // compute units of the device
    void* pts = nullptr;     // [npad][stride] of float or double
    // per-point nearest-neighbour squared distances (unscaled), min over j != i,
    // in x and in y separately; computed once, used as the grid kernel's shifts
    void* nn = nullptr;      // [2][npad] doubles (FP32 models, grid path)
    bool nn_ready = false;
    void* xmean = nullptr;   // [16] floats: column means of x (cross-term option)
    bool xmean_ready = false;
    // spatial order (compact-support kernels; built on first use)
    void* spts = nullptr;    // [npad][stride] doubles: rows in Morton order of x
    void* perm = nullptr;    // [npad] ints: sorted position -> original index
    void* tbox = nullptr;    // [npad/TILE][2][dx] doubles: x box of each sorted tile
    void* sbox = nullptr;    // [npad/SUBROWS][2][dx] doubles: x box of each sorted subtile
    bool index_ready = false;
    void* scratch = nullptr; // block partials and flags
    size_t scratch_bytes = 0;
    size_t bytes = 0;
    // Data extent (per-dimension minimum and maximum of the training set and
    // a non-finite flag), computed on the device by cde_create and copied to
    // pinned host memory; read once, at the first call that checks
    // bandwidths (ext_event marks the copy's completion).
    unsigned long long* ext_dev = nullptr;   // [2 * MAXP + 1], in the tail of pts
    unsigned long long* ext_host = nullptr;  // pinned copy
    hipEvent_t ext_event = nullptr;
    bool ext_known = false;
    bool data_finite = true;
    double range[cde::MAXP] = {};            // max - min per dimension
    // Grouped grid evaluation (cde_launch_batch) in progress: the next point
    // range must start at batch_next (0: none in progress), for the grid and
    // criterion whose signature is batch_sig.
    int64_t batch_next = 0;
    uint64_t batch_sig = 0;
};
