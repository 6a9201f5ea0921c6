// Internal declarations shared by the kernels and the host runtime of libqsw.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsw {

constexpr int kMMax = 55;   // largest Taylor degree
constexpr int kPMax = 8;    // largest p in alpha_p = max(d_p, d_{p+1})
constexpr int kMaxBlockPoints = 4096;  // time-series block length handled per launch chain

// Norm slots of one scaling step of the single-time algorithm.  Maxima of
// non-negative doubles are kept as their IEEE bit patterns, whose unsigned
// order equals the numeric order (NaN sorts above +inf).
struct StepSlots {
  unsigned long long b0;               // ||b||_inf at the start of the step
  unsigned long long b[kMMax + 1];     // ||b_j||_inf after term j
  unsigned long long f[kMMax + 1];     // ||F||_inf after term j
  int stop;                            // set once the two-term test has passed
  int pad[3];
};

// Per-block state of the time-series algorithm (stored powers branch).
struct SeriesSlots {
  unsigned long long kn[kMMax + 1];    // ||K_p||_inf, K_0 = Z
  int mhat;                            // powers K_1..K_mhat already formed
  int pad[3];
};

struct DeviceState {
  StepSlots step[2];                   // alternating per scaling step
  SeriesSlots series;
  unsigned long long products;         // sparse products computed
  int nonfinite;
  int pad[3];
};

// Per point k of a series block: ||F_k||_inf after term p, and the stop flag.
struct PointSlots {
  unsigned long long f[kMMax + 1];
  int stop;
  int pad[3];
};

struct AssembleArgs {
  int32_t N;
  const int64_t *hp;     // off-diagonal H, CSR over N rows
  const int32_t *hc;
  const double2 *hv;
  const double *hdiag;   // H_aa (real: H is Hermitian)
  const int64_t *rp;     // off-diagonal rates, CSR over N rows (row a: entries (a, j))
  const int32_t *rc;
  const double *rv;
  const double *rdiag;   // R_aa
  const double *K;       // K_j = sum_i R_ij of the ORIGINAL rates
  const int64_t *PH;     // exclusive prefix sums of the off-diagonal H row counts
  const int64_t *PR;     // exclusive prefix sums of the off-diagonal rate row counts
  int64_t EH;            // off-diagonal H entries
  double omega;
  double sigma;          // +1: L ; -1: L^dagger (with R transposed)
  int64_t *row_ptr;
  int32_t *col;
  double2 *val;
};

struct SpmvArgs {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const double2 *val;
  const double2 *x;      // gathered vector
  const double2 *fin;    // accumulator in (Taylor mode)
  double2 *fout;         // accumulator out (may equal fin)
  double2 *y;            // output term
  double alpha;          // scale of the product
  double tol;
  DeviceState *st;
  int par;               // scaling-step parity
  int j;                 // term index (1-based)
  int64_t rows_per_block;// contiguous rows handled by one workgroup
};

// ---- launchers (kernels.hip) ----
hipError_t launch_assemble(const AssembleArgs &a, int64_t n, hipStream_t s);
hipError_t launch_row_abs_max(int64_t n, const int64_t *rp, const double2 *val,
                              unsigned long long *out_bits, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_copy(double2 *dst, const double2 *src, int64_t n, hipStream_t s);

// Single-time algorithm term j: y = alpha A x; F_out = F_in + y; norms into
// st->step[par]; early exit when the previous terms already passed the test.
hipError_t launch_taylor_term(const SpmvArgs &a, int lpr, int grid, hipStream_t s);

// y = alpha A x (no accumulation, no norms).
hipError_t launch_spmv(const SpmvArgs &a, int lpr, int grid, hipStream_t s);

// Time-series branch.
hipError_t launch_series_init(DeviceState *st, PointSlots *pts, int npts,
                              const double2 *Z, int64_t n, int grid, hipStream_t s);
hipError_t launch_series_power(const SpmvArgs &a, PointSlots *pt, int k, int p,
                               int lpr, int grid, hipStream_t s);
hipError_t launch_series_accum(DeviceState *st, PointSlots *pt, int k, int p,
                               const double2 *Kp, const double2 *Z, double2 *F,
                               int64_t n, double tol, int grid, hipStream_t s);

// Block 1-norm estimation helpers (two right-hand sides, interleaved rows).
// mode 0: Y = A X; mode 1: Y = A X, column |.|_1 partials per block into
// part[2*block + c] and S = sign(Y) into sgn; mode 2: Y = A X and
// h[i] = max_c |Y[i][c]|.
hipError_t launch_spmm2(int64_t n, const int64_t *rp, const int32_t *col,
                        const double2 *val, const double2 *X, double2 *Y, int mode,
                        double *part, double2 *sgn, double *h, int grid,
                        hipStream_t s);
// Number of workgroups launch_spmm2 uses for (n, grid): the length of part[]/2.
int spmm2_blocks(int64_t n, int grid);
hipError_t launch_sum_partials(const double *part, int nblocks, double *out2,
                               hipStream_t s);

hipError_t launch_populations(const double2 *rho, int32_t N, int32_t count, double *pops,
                              hipStream_t s);

}  // namespace qsw
