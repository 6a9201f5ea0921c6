// Internal declarations shared by the kernels and the host runtime of libqsw.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsw {

constexpr int kMMax = 55;   // largest Taylor degree
constexpr int kPMax = 8;    // largest p in alpha_p = max(d_p, d_{p+1})
#ifndef QSW_BLOCK
#define QSW_BLOCK 256
#endif
constexpr int kBlockThreads = QSW_BLOCK;  // threads per workgroup of the product kernels
constexpr int kCap = QSW_BLOCK * 8;       // LDS product slots per workgroup (8 entries per lane)
constexpr int kTopKMax = 16;  // candidates the 1-norm estimator ranks at once

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
  // single-precision products (QSW_PREC_FP32): the trace check of each
  // output point in double
  double tr0;                          // Tr rho0 (after exp(t0 L), the reference)
  double scale;                        // factor of the point being written
  unsigned long long trace_dev;        // max |Tr rho_k - tr0| before the factor (bits)
  unsigned long long pad2;
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
  double omega;          // H terms carry 1 - omega
  double rscale;         // factor on the rates, K and R_aa (omega, or 1 when pre-scaled)
  double sigma;          // +1: L ; -1: L^dagger (with R transposed)
  int64_t *row_ptr;
  int32_t *col;
  double2 *val;
};

// Wave-jagged execution layout: rows in blocks of 64 (one wavefront each).
// Inside a block the rows are ranked by length (longest first, ties by row)
// and the stored entries placed position-major: entry p of the row of rank r
// sits at wstart[k] + (stored entries of positions < p) + r.  wlen[64 k + r]
// is the length of the row of rank r (shared positions included) and
// wperm[64 k + r] its index within the block.
constexpr int kWaveRows = 64;
// wglob[k]: G | kGlobDiagFirst when position G holds every row's diagonal
constexpr int32_t kGlobDiagFirst = 1 << 30;
constexpr int32_t kGlobMask = kGlobDiagFirst - 1;
constexpr int kWavePad = 64;  // zero entries after the wave-jagged arrays (reads past a block's end)
constexpr size_t kStageMaxBytes = 32768;  // largest LDS-staged rho-row (N <= 2048)
// Stored entries per row (on average) from which a staged handle takes the
// wide-group traversal (engine 300): the 1024-vertex benchmark operator has
// 21, the complete graph of 400 vertices about 740.
constexpr int64_t kWideRowEntries = 128;

// The wave layout stores each entry's column as its offset from the entry's
// row (column - row), so that blocks whose rows have the same pattern and
// values relative to themselves store the same words.
// Phase-split values.  Every off-diagonal entry of a graph-built L-QSW
// superoperator is real (the rate terms) or imaginary (the Hamiltonian
// terms): such an entry is stored as one real coefficient c, with the phase
// (1 or i) in the top bit of its column word and the offset in the low 30
// bits (two's complement).  The diagonal entry of each row is complex; it
// keeps its place in the row (flag kDiagBit) and its value is read from a
// per-row array.  Offsets then need n <= 2^29.
constexpr uint32_t kImagBit = 0x80000000u;  // value i c
constexpr uint32_t kDiagBit = 0x40000000u;  // value wdiag[row]
constexpr uint32_t kOffMask = 0x3fffffffu;
constexpr int64_t kSplitMaxN = (int64_t)1 << 29;

// Block-shared positions (phase-split layouts).  When every row of a 64-row
// block has, at leading position p, an entry at the same offset from its own
// row (column = row + off) with the same value (as the H rho part does: all
// rows of a block share their rho-row a, and entry p is c_p N + b with value
// -i (1 - omega) H_a,c_p), the position is stored once for the block instead
// of once per row.  A block's shared positions are padded with zero entries
// (off 0, value 0) to a multiple of kSharedPad.
struct SharedEntry {
  int32_t off;     // column - row
  uint32_t flags;  // kImagBit: value i coef
  double coef;
};
constexpr int kSharedPad = 8;
// At most this many leading positions of a block are shared, so a block's
// shared entries are one load per lane and sit at a fixed stride (a block
// with more keeps the rest in its rows).
constexpr int kSharedMax = 64;
static_assert(sizeof(SharedEntry) == 16, "a shared entry is read as one 16-byte load");

struct SpmvArgs {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const double2 *val;
  // stream engine: row blocks blk[0..nblk] (block k = rows blk[k]..blk[k+1]-1),
  // each workgroup takes blocks_per_wg consecutive blocks
  const int32_t *blk;
  int32_t nblk;
  int32_t blocks_per_wg;
  // vector engine: contiguous rows per workgroup
  int64_t rows_per_block;
  // wave-jagged engine
  int32_t N;             // graph order (rho-row length for the staged engines)
  int64_t nwb;           // blocks of 64 rows
  const int32_t *wcol;
  const double2 *wval;
  const float2 *wval32;  // complex64 copy of wval (engine 1), or null
  const double *wcoef;   // phase-split values (engines +10): coefficient per entry
  const float *wcoef32;  //   its single-precision copy
  const double2 *wdiag;  //   diagonal value of the row of rank r at 64 k + r
  const float2 *wdiag32; //   its complex64 copy
  const int32_t *wlen;
  const unsigned char *wperm;
  const int32_t *wglob;  // per block: first position inside the rho-row, or -1 (may be null)
  const int64_t *wstart; // per block: first per-row entry (with shared positions), or null: rp
  const int32_t *wshn;   // per block: shared leading positions (null: none)
  const int64_t *wshs;   //   first shared entry of block k: k wsh_stride
  const SharedEntry *wsh;
  int32_t wsh_stride;    //   entries per block (a multiple of kSharedPad, <= kSharedMax)
  const double2 *x;      // gathered vector (NRHS interleaved columns for the estimator)
  const double2 *fin;    // accumulator in (Taylor mode)
  double2 *fout;         // accumulator out (may equal fin)
  double2 *y;            // output term
  double alpha;          // scale of the product
  double tol;
  DeviceState *st;
  int par;               // scaling-step parity
  int j;                 // term index (1-based)
  // paced launches (null progress: none): launch number seq posts
  // ((seq - 1) << 1) | (the step passed its test after launch seq - 1) to
  // this host-visible word
  unsigned long long *progress;
  unsigned long long seq;
  // single-precision products (QSW_PREC_FP32): complex64 x and term, and the
  // accumulator as a two-float (hi + lo) pair of complex64 vectors
  const float2 *x32;
  float2 *y32;
  const float2 *fin_hi, *fin_lo;
  float2 *fout_hi, *fout_lo;
  // products with L^dagger through the phase-split layout of L (graph walks
  // with a real H; the estimator's adjoint products): Hamiltonian entries
  // negated, the diagonal conjugated, the real off-diagonal entries (the
  // population transfers of the rows (a, a)) dropped and L^dagger's own
  // added from the transposed rates: row a of trp / tcol / tval holds
  // omega R_ja for rho_jj, ascending j
  int32_t adj_fwd;
  int32_t adj_grid;  // (set by the launch) workgroups taking blocks; the rest take the rows (a, a)
  const int64_t *trp;
  const int32_t *tcol;
  const double *tval;
};

// ---- batched propagation (several walks advance together) ----
constexpr int kBatchMaxRhs = 4;

enum BatchOpType : int32_t {
  BOP_NONE = 0,   // nothing this cycle (finished, or waiting)
  BOP_LOAD = 1,   // V[0] = rho0 (interleaved, zero columns beyond n0)
  BOP_TERM = 2,   // Taylor term: y = alpha A x, fout = fin + y on active columns
  BOP_POWACC = 3, // series power y = K_p = alpha A K_{p-1}, fout = fin + k^p y
  BOP_ACC = 4,    // series accumulation from a stored power: fout = fin + k^p K_p
  BOP_NORM = 5,   // series block start: max |Z| per column
  BOP_EMIT = 6,   // out / pops of one grid point from x
  BOP_TRACE = 7   // single-precision products: trace of the state pair per column
                  // (first: the reference; else the check's scale factor)
};

// One walk in the batch (fixed while it runs).  Vectors hold R complex128
// columns one after the other: element (row, c) at c * n + row.
struct BatchInst {
  const int64_t *rp;
  const int32_t *wcol;
  const double2 *wval;
  const float2 *wval32;
  const double *wcoef;
  const float *wcoef32;
  const double2 *wdiag;
  const float2 *wdiag32;
  const int32_t *wlen;
  const unsigned char *wperm;
  const int64_t *wstart;
  const int32_t *wshn;
  const int64_t *wshs;
  const SharedEntry *wsh;
  int32_t wsh_stride;
  int64_t n, nwb;
  int64_t vlen;      // n * R: complex elements of one work vector
  int32_t N, f32, split;  // f32: single-precision values; split: phase-split values
  // plan (as for one walk)
  int32_t branch, m, s, m0, s0, d, jb, r, q, n0;
  double t0, dt, tol;
  double2 *V[2], *F[2], *B[2];
  double2 *K;        // m stored powers (series branch)
  double *kn;        // (m + 1) x 4 power norms (series branch)
  const double2 *rho0;
  double2 *out;
  double *pops;
  // single-precision products (prec32): the state and accumulator as hi + lo
  // pairs of complex64 vectors (pair c: Ph[c], Pl[c]; the state is pair
  // `cur`, each scaling step accumulates into the other), complex64 terms
  int32_t prec32;
  float2 *Ph[2], *Pl[2], *B32[2];
};

struct BatchOp {
  int32_t type;
  uint32_t active;   // columns whose accumulator is updated
  int32_t first;     // TERM: j == 1; POWACC / ACC: p == 1
  int32_t point;     // EMIT: grid point
  double alpha, kpow;
  const double2 *x;
  double2 *y;
  const double2 *fin;
  double2 *fout;
  // single-precision products: TERM x32, y32 and the accumulator pairs;
  // TRACE and EMIT: the state pair (fout_hi, fout_lo)
  const float2 *x32;
  float2 *y32;
  const float2 *fin_hi, *fin_lo;
  float2 *fout_hi, *fout_lo;
};

struct BatchCtl {
  int32_t pc, cur, i, j, mseg, sseg, seg, point;
  int32_t blk, dd, zi, kk, p, mhat;
  uint32_t active;
  int32_t last;      // type of the op in flight
  int32_t done;
  int32_t nonfinite;
  int64_t products;
  double tseg;
  double c_prev[kBatchMaxRhs], c_last[kBatchMaxRhs], f_last[kBatchMaxRhs];
  unsigned long long trace_dev;  // largest |Tr - Tr rho0| seen (bits; single-precision products)
};

struct BatchSlots {  // maxima of the op in flight, as IEEE bit patterns
  unsigned long long y[kBatchMaxRhs], f[kBatchMaxRhs], b0[kBatchMaxRhs];
  // single-precision products: per column the reference trace and the
  // scale factor of the last check, and the largest deviation of the last
  // check (bits)
  double tr0[kBatchMaxRhs], scale[kBatchMaxRhs];
  unsigned long long trace_dev;
};

struct BatchArgs {
  const BatchInst *inst;
  BatchCtl *ctl;
  BatchOp *op;
  BatchSlots *slots;
  const int32_t *act;        // active instance ids, nact of them
  const int64_t *blk_start;  // nact + 1 prefix of their wave blocks
  int2 *blkmap;              // per global block: (instance id, block within it)
  int64_t nblocks;           // blk_start[nact]
  int32_t stage_bytes;       // dynamic LDS for the rho-row of R columns (0: no staging)
  int32_t nact, count;
  unsigned int *live;        // control: instances not finished
  int *nonfinite;
};

// ---- launchers (kernels.hip) ----
hipError_t launch_assemble(const AssembleArgs &a, int64_t n, hipStream_t s);
hipError_t launch_row_abs_max(int64_t n, const int64_t *rp, const double2 *val,
                              unsigned long long *out_bits, hipStream_t s);
// The same maximum (||L||_1) from the CSR of L of a graph walk with a real
// H, without the CSR of L^dagger: frp is the row pointer of L's rates, trp /
// tval the transposed rates' (omega R_ja in row a); bit for bit the value of
// launch_row_abs_max on L^dagger's CSR.
hipError_t launch_adj_row_abs_max(int64_t n, int32_t N, const int64_t *rp, const double2 *val,
                                  const int64_t *frp, const int64_t *trp, const double *tval,
                                  unsigned long long *out_bits, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_copy(double2 *dst, const double2 *src, int64_t n, hipStream_t s);
hipError_t launch_to_c64(float2 *dst, const double2 *src, int64_t n, hipStream_t s);
hipError_t launch_to_f32(float *dst, const double *src, int64_t n, hipStream_t s);

// Stream-engine row blocks: block k starts at the first row whose first
// entry index is >= k B; blk has nblk + 1 entries.
hipError_t launch_row_blocks(const int64_t *rp, int64_t n, int64_t B, int32_t *blk, int64_t nblk,
                             hipStream_t s);

// Wave-jagged layout of a CSR (n rows, graph order N), one wavefront per
// 64-row block; inside each row the entries outside the row's rho-row first.
// Plan: wglob[k] (the position G at which every row of block k passes from
// entries outside its rho-row to entries inside it, when all its rows share
// one rho-row and such a G exists; else -1), wshn[k] (shared leading
// positions; 0 unless `shared`, which needs phase-split values) and wcnt[k]
// (per-row entries of the block after them).
hipError_t launch_wjag_plan(const int64_t *rp, const int32_t *col, const double2 *val, int64_t n,
                            int32_t N, bool shared, int32_t *wglob, int32_t *wshn, int64_t *wcnt,
                            hipStream_t s);
// Fill, from the plan's prefix sums wstart (per-row entries) and wshs
// (padded shared entries): complex values (wval) unless `split`, then
// phase-split values (wcoef per entry, wdiag per row, zero for a row without
// a diagonal entry; *bad, zeroed by the caller, is set when an off-diagonal
// entry has a non-zero real and imaginary part or a row holds its diagonal
// more than once).
hipError_t launch_wjag_fill(const int64_t *rp, const int32_t *col, const double2 *val, int64_t n,
                            int32_t N, bool split, const int32_t *wshn, const int64_t *wstart,
                            const int64_t *wshs, int32_t *wcol, double2 *wval, double *wcoef,
                            double2 *wdiag, int32_t *wlen, unsigned char *wperm, SharedEntry *wsh,
                            int *bad, hipStream_t s);

// Block dedup: hash[k] of block k's stored rows (lengths after the shared
// positions and its words from wstart[k] to wstart[k+1]); same[k] = 1 when
// they equal those of block canon[k] (0 for canon[k] == k).
hipError_t launch_wjag_hash(const int32_t *wcol, const double *wcoef, const double2 *wval,
                            const int32_t *wlen, const int32_t *wshn, const int64_t *wstart,
                            int64_t n, unsigned long long *hash, hipStream_t s);
hipError_t launch_wjag_same(const int32_t *wcol, const double *wcoef, const double2 *wval,
                            const int32_t *wlen, const int32_t *wshn, const int64_t *wstart,
                            int64_t n, const int64_t *canon, int *same, hipStream_t s);

// Engine: wave-jagged traversal 0 (plain), 100 (rho-row staged in LDS) or
// 200 (staged, XCD-banded), plus 1 for single-precision values and 10 for
// phase-split values; 3 = CSR stream; 4/8/16/32/64 = vector with that many
// lanes per row.
// Single-time algorithm term j: y = alpha A x; F_out = F_in + y; norms into
// st->step[par]; early exit when the previous terms already passed the test.
hipError_t launch_taylor_term(const SpmvArgs &a, int engine, int grid, hipStream_t s);

// The same with complex64 vectors and single-precision products (engines
// 1, 11, 101, 111; a.x32, a.y32, a.fin_hi/lo, a.fout_hi/lo): the term y32 =
// alpha A x32 is rounded once from the float row sum scaled in double, and
// F = F_in + y32 is kept as an unevaluated hi + lo pair of floats.
hipError_t launch_taylor_term32(const SpmvArgs &a, int engine, int grid, hipStream_t s);
// hi + lo = v for n complex128 elements (hi the nearest float, lo the nearest
// float to the remainder).
hipError_t launch_split_c64(const double2 *v, float2 *hi, float2 *lo, int64_t n, hipStream_t s);
// Trace check of a two-float density matrix (N x N): tr = sum_a (hi + lo)_aa
// in double; reference = 1 stores it as st->tr0, else st->scale = tr0 / tr
// (1 when either is zero or not finite, or |tr - tr0| > 2^-10 |tr0|) and
// st->trace_dev = max(., |tr - tr0|).
hipError_t launch_trace32(DeviceState *st, const float2 *hi, const float2 *lo, int32_t N,
                          int reference, hipStream_t s);
// out = (hi + lo) st->scale in complex128, and hi, lo re-split from it.
hipError_t launch_emit32(const DeviceState *st, float2 *hi, float2 *lo, double2 *out, int64_t n,
                         hipStream_t s);

// y = alpha A x (no accumulation, no norms).
hipError_t launch_spmv(const SpmvArgs &a, int engine, int grid, hipStream_t s);

// Time-series branch.
hipError_t launch_series_init(DeviceState *st, PointSlots *pts, int npts,
                              const double2 *Z, int64_t n, int grid, hipStream_t s);
hipError_t launch_series_power(const SpmvArgs &a, PointSlots *pt, int k, int p,
                               int engine, int grid, hipStream_t s);
hipError_t launch_series_accum(DeviceState *st, PointSlots *pt, int k, int p,
                               const double2 *Kp, const double2 *Z, double2 *F,
                               int64_t n, double tol, int grid, hipStream_t s);

// Block 1-norm estimation helpers: Y = A X for two interleaved right-hand
// sides (wave-jagged engine; a.x = X, a.y = Y).  mode 0: product only; mode 1:
// also column |.|_1 partial sums per workgroup into part[2*wg + c] and
// S = sign(Y) into sgn; mode 2: also h[i] = max_c |Y[i][c]|.
// split: the layout holds phase-split values.
hipError_t launch_spmm2(const SpmvArgs &a, bool split, int mode, double *part, double2 *sgn,
                        double *h, int grid, hipStream_t s);
hipError_t launch_sum_partials(const double *part, int nblocks, double *out2,
                               hipStream_t s);

// Several estimates at once.  The power chains of the estimates of ||A^p||_1
// for different p (two columns each) advance together: step i applies A (or
// A^dagger) to the columns of every chain with p >= i, held interleaved
// (element (row, c) at row nr + c, chains by decreasing p), so one pass over
// the matrix serves them all.  The chain with p = i (the last pair of
// columns) finishes at step i; its epilogue is the two-column product's.
constexpr int kEstChainsMax = kPMax;  // estimates of p = 2 .. kPMax + 1
constexpr size_t kEstWideBytes = (size_t)4 << 30;  // largest wide block (three are held)
constexpr int64_t kEstMergeMaxN = (int64_t)1 << 16;  // merged by default up to this many rows
struct WideOut {
  double2 *Y;     // continuing columns: Y[row ys + c], c < ys
  int ys;         // nr - 2 fin
  int fin;        // the last pair finishes at this step
  int mode;       // 1: column sums and sign block; 2: row maxima (of the last pair)
  double2 *sgn;   // mode 1: sign block of the last pair (n x 2 interleaved)
  double *h;      // mode 2: h[row] = max |Y_row,c| over the last pair
  double *part;   // mode 1: per-workgroup column sums of the last pair (2 per workgroup)
};
// nr = 2 .. 2 kEstChainsMax, even; a.x holds the nr interleaved columns.
hipError_t launch_spmm_wide(const SpmvArgs &a, bool split, int nr, const WideOut &o, int grid,
                            hipStream_t s);
// W[row c + 2 j + q] = src[j][2 row + q] (j < chains, q < 2; c = 2 chains).
struct PairSources {
  const double2 *src[kEstChainsMax];
  int chains;
};
hipError_t launch_pack_pairs(double2 *W, int64_t n, const PairSources &ps, hipStream_t s);
// W[row c + 2 j + q] = 1 where row = ind[j][q] (ind < 0: none), else 0.
struct PairUnits {
  int64_t ind[kEstChainsMax][2];
  int chains;
};
hipError_t launch_unit_pairs(double2 *W, int64_t n, const PairUnits &pu, hipStream_t s);
// Estimator probe block (column 0 = 1/n, column 1 = signed 1/n; t = 1 zeroes
// column 1), unit columns [e_i0, e_i1] (i1 < 0: zero), and the top K <= 16
// of h by (larger value, then smaller index) through grid * K candidates.
hipError_t launch_probe_init(double2 *X, int64_t n, int t, hipStream_t s);

// A few results of the 1-norm estimator posted to pinned host memory: the
// values, the indices, then the sequence number with a system-scope release
// store, on which the host waits instead of synchronising the stream.
constexpr int kPostMax = kEstChainsMax * (kTopKMax + 1);
struct HostPost {
  double v[kPostMax];
  int64_t i[kPostMax];
  unsigned long long seq;
};
static_assert(kTopKMax + 1 <= kPostMax, "the top-k values and one more fit");
// dst->v[0 .. nv) = v, dst->i[0 .. ni) = iv, dst->v[nv] = *extra (if given),
// then dst->seq = seq; nv + 1, ni <= kPostMax.
hipError_t launch_post(const double *v, int nv, const int64_t *iv, int ni, const double *extra,
                       HostPost *dst, unsigned long long seq, hipStream_t s);
// Several chains' results in one post: chain j's nv[j] values at
// dst->v[j (kTopKMax + 1)], then *extra[j] (if given), and its ni[j] indices
// at dst->i[j kTopKMax]; nv[j] + 1, ni[j] <= kTopKMax + 1.
struct PostList {
  const double *v[kEstChainsMax];
  const int64_t *i[kEstChainsMax];
  const double *extra[kEstChainsMax];
  int nv[kEstChainsMax];
  int ni[kEstChainsMax];
  int chains;
};
hipError_t launch_post_list(const PostList &l, HostPost *dst, unsigned long long seq,
                            hipStream_t s);
hipError_t launch_unit_cols(double2 *X, int64_t n, int64_t i0, int64_t i1, hipStream_t s);
// dst = src (n x 2 interleaved) with its two columns exchanged; dst != src.
hipError_t launch_swap_pairs(double2 *dst, const double2 *src, int64_t n, hipStream_t s);
hipError_t launch_topk(const double *h, int64_t n, int K, int grid, double *cand_v, int64_t *cand_i,
                       double *out_v, int64_t *out_i, hipStream_t s);

// Workgroups of the product kernels that fit on the device at once
// (which = 0: wave layout, single right-hand side, 1: two; 2: the CSR
// stream engine).
int resident_workgroups(int which);
hipError_t launch_batch_control(const BatchArgs &a, hipStream_t s);
// The work kernel of the walks with double (p32 false) or single-precision
// (p32 true) products.
hipError_t launch_batch_work(const BatchArgs &a, int rhs, bool p32, int grid, hipStream_t s);
hipError_t launch_batch_blocks(const BatchArgs &a, hipStream_t s);
int batch_resident_workgroups(int rhs);

hipError_t launch_populations(const double2 *rho, int32_t N, int32_t count, double *pops,
                              hipStream_t s);

}  // namespace qsw
