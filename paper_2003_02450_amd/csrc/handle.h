// Host-side internals of libqsw shared by its runtime files: the
// superoperator handle, the plan of one propagation, small HIP helpers.
#pragma once

#include "qsw_impl.h"
#include "../../include/qsw.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdlib>
#include <memory>
#include <mutex>

namespace qsw {

struct Assembler;  // what a handle is built from (runtime.hip)

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return ::qsw::status_of(_e); \
  } while (0)

inline qsw_status_t status_of(hipError_t e) {
  if (e == hipSuccess) return QSW_OK;
  if (e == hipErrorOutOfMemory) return QSW_ERR_OOM;
  return QSW_ERR_DEVICE;
}

// Device memory of the library (handle arrays and build temporaries).  A
// freed block is kept, per device and size, for the next allocation of the
// same size (repeated builds ask for the same sizes), up to QSW_POOL_MB
// megabytes (default 16384; 0: free at once).  Before it keeps a block the
// pool waits for the device to finish its work, as hipFree would.  When
// hipMalloc fails, the device's kept blocks are released and it is retried.
hipError_t pool_alloc(void **p, size_t bytes);
void pool_free(void *p);

template <class T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return pool_alloc((void **)p, count * sizeof(T));
}

template <class T>
void dfree(T *&p) {
  if (p) pool_free((void *)p);
  p = nullptr;
}

// Save and restore the caller's current device around an API call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline int env_int(const char *name, int dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace qsw

// The handle behind qsw_superop_t.

struct qsw_superop_s {
  int device = -1;
  int32_t N = 0;
  int64_t n = 0, nnz = 0;
  double omega = 0.0;
  int64_t *row_ptr = nullptr;
  int32_t *col = nullptr;
  double2 *val = nullptr;
  qsw_info_t info{};
  // launch shape of the product kernels
  int engine = 0;                 // wave-jagged traversal 0 / 100 (rho-row staged in
                                  // LDS) / 200 (staged, XCD-banded); 3: CSR stream;
                                  // 4..64: vector engine lanes per row
  int grid = 0;                   // workgroups of a product launch
  int64_t rows_per_block = 0;     // vector engine
  int32_t *blk = nullptr;         // stream engine row blocks
  int32_t nblk = 0;
  int32_t blocks_per_wg = 0;
  // wave-jagged layout (the product kernels' copy of the matrix)
  int32_t *wcol = nullptr;
  double2 *wval = nullptr;        // complex values (null with phase-split values)
  float2 *wval32 = nullptr;       // complex64 values for QSW_PREC_SINGLE propagation
  bool split = false;             // phase-split values: wcoef / wdiag instead of wval
  double *wcoef = nullptr;
  float *wcoef32 = nullptr;       // single-precision copies for QSW_PREC_SINGLE
  double2 *wdiag = nullptr;
  float2 *wdiag32 = nullptr;
  int prec = QSW_PREC_DOUBLE;     // precision of qsw_propagate
  int32_t *wlen = nullptr;
  unsigned char *wperm = nullptr;
  int32_t *wglob = nullptr;       // per block: where its rows leave the gathers outside the rho-row
  int32_t *wshn = nullptr;        // per block: shared leading positions
  int64_t *wstart = nullptr;      // per block: first per-row entry
  int64_t *wshs = nullptr;        // per block: first shared entry (padded prefix)
  qsw::SharedEntry *wsh = nullptr;
  int32_t wsh_stride = 0;         // shared entries of block k at wsh + k wsh_stride
  int64_t wentries = 0;           // per-row entries stored
  int64_t wshared = 0;            // shared entries stored (padded)
  int64_t wdistinct = 0;          // per-row entries in the copies the blocks read
  int64_t nwb = 0;
  // last propagate
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  unsigned long long *stats_dev = nullptr;  // [products, nonfinite]
  qsw_stats_t last{};
  bool last_fused = false;  // the last series call ran one-point blocks in the term kernel
  bool have_last = false;
  std::shared_ptr<qsw::Assembler> src;  // kept for qsw_superop_set_omega
  // paced term launches (qsw_superop_set_pacing): at most `pace` ahead of the
  // device; the device posts progress to a pinned host word
  int pace = 0;
  unsigned long long *pace_host = nullptr;  // pinned, coherent
  unsigned long long *pace_dev = nullptr;   // its device address
  unsigned long long pace_seq = 0;          // last paced launch number
  std::unique_ptr<std::mutex> pace_mu;
};

namespace qsw {

inline bool is_wave_engine(int engine) {
  return engine == 0 || engine == 100 || engine == 200 || engine == 300;
}

// Kernel engine of a product launch: the handle's traversal plus its value
// format (+10 phase-split, +1 single precision when `single`).
inline int launch_engine(const qsw_superop_s *h, bool single) {
  if (!is_wave_engine(h->engine)) return h->engine;
  // wide groups serve double values; single-precision values and products
  // take the plain staged traversal
  const int base = (single && h->engine == 300) ? 100 : h->engine;
  return base + (h->split ? 10 : 0) + (single ? 1 : 0);
}

// Parameters and workspace layout of one qsw_propagate call.
struct Plan {
  int branch = 0;
  int m = 0, s = 1;      // per interval (branch 0) or for the span (branch 1)
  int m0 = 0, s0 = 1;    // exp(t0 L) start
  int d = 0, j = 0, r = 0;
  size_t off_state = 0, off_pts = 0, off_B = 0, off_F = 0, off_K = 0, total = 0;
};

// (m, s) and the branch for rho(t0 + k dt), k = 0..n_steps, from the handle's
// norms at its precision (runtime.hip).
qsw_status_t make_plan(const qsw_superop_s *h, double t0, double dt, int32_t n_steps, Plan &P);

// Bytes of an engine's arena available to walks' vectors (batch.hip).
size_t engine_pool_bytes(const qsw_engine_s *e);

}  // namespace qsw
