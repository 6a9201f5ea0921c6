// HIP kernels of libqsw for gfx950 (MI355X): superoperator assembly, the
// complex128 CSR product with the fused Taylor-term epilogue, the
// time-series kernels and the block 1-norm estimation helpers.
//
// Two row engines compute the CSR product; both feed the same epilogues.
//  * stream: a workgroup takes row blocks of at most kCap entries, streams
//    their values and column indices with fully coalesced loads (a wave
//    reads 64 consecutive entries per instruction, several loads in flight
//    per lane), gathers x, stages the products in LDS and then reduces each
//    row with a power-of-two group of lanes in a fixed order.  Contiguous
//    runs of blocks are given to the workgroups of one XCD.
//  * vector: LPR lanes per row stride through the row (kept for tuning and
//    for comparison).
// Every reduction order is fixed by the matrix, so results are bitwise
// reproducible.
//
// Maxima of non-negative doubles travel as IEEE bit patterns in 64-bit
// unsigned integers: their unsigned order is the numeric order, so a plain
// integer atomicMax merges them independently of workgroup order, and NaN
// (after fabs) sorts above +inf, so a non-finite value reaches the slots.
#include "qsw_impl.h"

#include <hip/hip_runtime.h>

#include <type_traits>

namespace qsw {

namespace {

constexpr int kBlock = kBlockThreads;
constexpr int kWaves = kBlock / 64;
constexpr int kUnroll = 8;  // independent entries in flight per lane (stream engine)

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ double bits_to_d(unsigned long long u) {
  return __longlong_as_double((long long)u);
}
__device__ __forceinline__ double cabs2(double2 z) { return sqrt(fma(z.x, z.x, z.y * z.y)); }

__device__ __forceinline__ unsigned long long umax(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_umax(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = umax(v, __shfl_xor(v, off, 64));
  return v;
}

constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

// Reduce NV maxima over the workgroup and merge them into dst[] with one
// atomic each; a maximum at or above +inf sets *nonfinite.  Every thread of
// the workgroup must call it.
template <int NV>
__device__ __forceinline__ void block_umax_to(unsigned long long (&v)[NV],
                                              unsigned long long *const (&dst)[NV],
                                              int *nonfinite) {
  __shared__ unsigned long long sm[NV][kWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    unsigned long long r = wave_umax(v[i]);
    if (lane == 0) sm[i][w] = r;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    unsigned long long m = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) m = umax(m, sm[threadIdx.x][k]);
    if (dst[threadIdx.x]) atomicMax(dst[threadIdx.x], m);
    if (nonfinite && m >= kInfBits) *(volatile int *)nonfinite = 1;
  }
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Every device pointer here addresses global memory.  A pointer the compiler
// cannot trace to a kernel argument (one read from memory, as in the batched
// kernels) would otherwise be accessed with generic (flat) instructions, which
// wait on both the vector-memory and the LDS counters; these helpers access
// through the global address space.
#define QSW_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gld(const T *p) {
  return *(const QSW_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ void gst(T *p, const T &v) {
  *(QSW_GLOBAL T *)p = v;
}
// double2's copy and assignment are member functions (generic `this`), so
// complex values travel as plain two-double vectors.
template <>
__device__ __forceinline__ double2 gld<double2>(const double2 *p) {
  const dvec2 v = *(const QSW_GLOBAL dvec2 *)p;
  return make_double2(v.x, v.y);
}
template <>
__device__ __forceinline__ void gst<double2>(double2 *p, const double2 &v) {
  dvec2 w;
  w.x = v.x;
  w.y = v.y;
  *(QSW_GLOBAL dvec2 *)p = w;
}

// Matrix entries of the wave layout.  Blocks with equal stored rows share
// one copy, which many blocks of a product read again, so these are plain
// (cached) loads: with non-temporal hints a product on the 1024-vertex
// operator took 8 % longer (at about the same L2 traffic).
__device__ __forceinline__ double2 load_entry(const double2 *p) { return gld(p); }
__device__ __forceinline__ int load_entry(const int32_t *p) { return gld(p); }
__device__ __forceinline__ double load_entry(const double *p) { return gld(p); }
__device__ __forceinline__ double load_entry(const float *p) { return (double)gld(p); }

// Entries of the plain CSR (stream and vector engines), each read once per
// product: non-temporal loads leave the caches to the gathered vector.
__device__ __forceinline__ double2 load_csr(const double2 *p) {
  const dvec2 v = __builtin_nontemporal_load((const QSW_GLOBAL dvec2 *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ int load_csr(const int32_t *p) {
  return __builtin_nontemporal_load((const QSW_GLOBAL int32_t *)p);
}

typedef float fvec2 __attribute__((ext_vector_type(2)));

// A block-shared entry as one 16-byte load.
template <>
__device__ __forceinline__ SharedEntry gld<SharedEntry>(const SharedEntry *p) {
  const dvec2 v = *(const QSW_GLOBAL dvec2 *)p;
  const unsigned long long head = (unsigned long long)__double_as_longlong(v.x);
  SharedEntry e;
  e.off = (int32_t)(uint32_t)head;
  e.flags = (uint32_t)(head >> 32);
  e.coef = v.y;
  return e;
}

template <>
__device__ __forceinline__ float2 gld<float2>(const float2 *p) {
  const fvec2 v = *(const QSW_GLOBAL fvec2 *)p;
  return make_float2(v.x, v.y);
}
template <>
__device__ __forceinline__ void gst<float2>(float2 *p, const float2 &v) {
  fvec2 w;
  w.x = v.x;
  w.y = v.y;
  *(QSW_GLOBAL fvec2 *)p = w;
}

// A complex64 entry widened to complex128 (exact).
__device__ __forceinline__ double2 load_entry(const float2 *p) {
  const float2 v = gld(p);
  return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ void cmac(double &ax, double &ay, double2 v, double2 x) {
  ax = fma(v.x, x.x, ax);
  ax = fma(-v.y, x.y, ax);
  ay = fma(v.x, x.y, ay);
  ay = fma(v.y, x.x, ay);
}
__device__ __forceinline__ double2 cmul(double2 v, double2 x) {
  return make_double2(fma(v.x, x.x, -v.y * x.y), fma(v.x, x.y, v.y * x.x));
}

// Single-precision products (complex64 vectors, single-precision values and
// sums): the same multiply-adds in float.
__device__ __forceinline__ void cmac(float &ax, float &ay, float2 v, float2 x) {
  ax = fmaf(v.x, x.x, ax);
  ax = fmaf(-v.y, x.y, ax);
  ay = fmaf(v.x, x.y, ay);
  ay = fmaf(v.y, x.x, ay);
}
__device__ __forceinline__ float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return fma(a, b, c); }

// Vector element and arithmetic types of a product: complex128 / double, or
// complex64 / float for the single-precision products (X32).
template <bool X32>
using VecT = std::conditional_t<X32, float2, double2>;
template <bool X32>
using RealT = std::conditional_t<X32, float, double>;

template <class V>
__device__ __forceinline__ V cplx(double re, double im);
template <>
__device__ __forceinline__ double2 cplx<double2>(double re, double im) {
  return make_double2(re, im);
}
template <>
__device__ __forceinline__ float2 cplx<float2>(double re, double im) {
  return make_float2((float)re, (float)im);
}
__device__ __forceinline__ float2 cplxf(float re, float im) { return make_float2(re, im); }
__device__ __forceinline__ double2 cplxf(double re, double im) { return make_double2(re, im); }

// The gathered vector of a product.
template <bool X32>
__device__ __forceinline__ const VecT<X32> *xbase(const SpmvArgs &a) {
  if constexpr (X32)
    return a.x32;
  else
    return a.x;
}

// --------------------------------------------------------------------------
// Row engines.  `epi(row, acc)` receives the complex sums of row `row` for
// NRHS right-hand sides (acc[2 r] = real, acc[2 r + 1] = imaginary part).
// --------------------------------------------------------------------------

// Logical workgroup index: the dispatcher deals workgroups to the 8 XCDs in
// turn, so regrouping gives each XCD one contiguous run of row blocks and
// keeps the vector slices those rows gather in that XCD's L2.
__device__ __forceinline__ int xcd_contiguous_index() {
  const int G = gridDim.x, w = blockIdx.x;
  if (G & 7) return w;
  return (w & 7) * (G >> 3) + (w >> 3);
}

// One row block of the stream engine.
struct BlockDesc {
  int64_t r0, r1;  // rows r0..r1-1
  int64_t e0;      // first entry
  int cnt;         // entries (valid when fits)
  bool fits;       // cnt <= stage capacity
};

__device__ __forceinline__ BlockDesc block_desc(const SpmvArgs &a, int64_t k, int cap) {
  BlockDesc d;
  d.r0 = a.blk[k];
  d.r1 = a.blk[k + 1];
  d.e0 = a.rp[d.r0];
  const int64_t c = a.rp[d.r1] - d.e0;
  d.fits = c <= cap && d.r1 - d.r0 <= cap;
  d.cnt = d.fits ? (int)c : 0;
  return d;
}

// Software-pipelined over the workgroup's run of blocks: while block k is
// reduced out of LDS, the column indices and values of block k+1 are
// already in flight.  Loads the reduction needs (row offsets, the
// epilogue's inputs) are issued before that prefetch, so waiting for them
// does not wait for it.
template <int NRHS, class Epi>
__device__ __forceinline__ void stream_engine(const SpmvArgs &a, Epi &epi) {
  constexpr int CAP = kCap / NRHS;  // entries staged per block
  static_assert(CAP <= kBlock * kUnroll, "one unrolled pass must cover a block");
  static_assert(kCap < 65536, "row offsets are stored in 16 bits");
  __shared__ double2 prod[kCap];
  __shared__ unsigned short rofs[kCap + 1];  // row starts of the block, relative to e0 (<= kCap)
  const int tid = threadIdx.x;
  int64_t k = (int64_t)xcd_contiguous_index() * a.blocks_per_wg;
  const int64_t kend = min((int64_t)a.nblk, k + a.blocks_per_wg);
  if (k >= kend) return;
  int c[kUnroll];
  double2 v[kUnroll];
  auto issue = [&](const BlockDesc &d) {
    const int32_t *cb = a.col + d.e0;
    const double2 *vb = a.val + d.e0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = tid + u * kBlock;
      if (i < d.cnt) {
        c[u] = load_csr(cb + i);
        v[u] = load_csr(vb + i);
      }
    }
  };
  BlockDesc cur = block_desc(a, k, CAP);
  if (cur.fits) issue(cur);
  while (k < kend) {
    if (cur.fits) {
      // descriptor of the next block first: its latency overlaps the gathers
      BlockDesc nxt{};
      nxt.fits = false;
      if (k + 1 < kend) nxt = block_desc(a, k + 1, CAP);
      // products of the staged block (x gathered) into LDS
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = tid + u * kBlock;
        if (i < cur.cnt) {
#pragma unroll
          for (int r = 0; r < NRHS; ++r)
            prod[i * NRHS + r] = cmul(v[u], a.x[(int64_t)c[u] * NRHS + r]);
        }
      }
      const int nr = (int)(cur.r1 - cur.r0);
      for (int i = tid; i <= nr; i += kBlock)
        rofs[i] = (unsigned short)(a.rp[cur.r0 + i] - cur.e0);
      int L = 64;
      while (L > 1 && nr * L > kBlock) L >>= 1;
      const int rpp = kBlock / L;
      const int g = tid / L, lane = tid & (L - 1);
      typename Epi::Pre pre{};
      if (g < nr && lane == 0) pre = epi.pre(cur.r0 + g);
      // next block's entries, in flight during this block's reduction
      if (nxt.fits) issue(nxt);
      __syncthreads();
      for (int base = 0; base < nr; base += rpp) {
        const int ri = base + g;
        double acc[2 * NRHS];
#pragma unroll
        for (int q = 0; q < 2 * NRHS; ++q) acc[q] = 0.0;
        if (ri < nr) {
          const int s = rofs[ri], t = rofs[ri + 1];
          for (int q = s + lane; q < t; q += L) {
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
              const double2 pv = prod[q * NRHS + r];
              acc[2 * r] += pv.x;
              acc[2 * r + 1] += pv.y;
            }
          }
        }
        for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
          for (int q = 0; q < 2 * NRHS; ++q) acc[q] += __shfl_xor(acc[q], off, L);
        }
        if (ri < nr && lane == 0) {
          if (base == 0) epi(cur.r0 + ri, acc, pre);
          else epi(cur.r0 + ri, acc, epi.pre(cur.r0 + ri));
        }
      }
      __syncthreads();
      cur = nxt;
      ++k;
    } else {
      // a block whose rows exceed the LDS stage: one row at a time, the
      // whole workgroup strides through it, fixed tree reduction
      double *red = reinterpret_cast<double *>(prod);
      for (int64_t row = cur.r0; row < cur.r1; ++row) {
        double acc[2 * NRHS];
#pragma unroll
        for (int q = 0; q < 2 * NRHS; ++q) acc[q] = 0.0;
        for (int64_t e = a.rp[row] + tid; e < a.rp[row + 1]; e += kBlock) {
          const double2 vv = a.val[e];
          const int64_t cc = a.col[e];
#pragma unroll
          for (int r = 0; r < NRHS; ++r)
            cmac(acc[2 * r], acc[2 * r + 1], vv, a.x[cc * NRHS + r]);
        }
#pragma unroll
        for (int q = 0; q < 2 * NRHS; ++q) red[q * kBlock + tid] = acc[q];
        __syncthreads();
        for (int w2 = kBlock / 2; w2 > 0; w2 >>= 1) {
          if (tid < w2) {
#pragma unroll
            for (int q = 0; q < 2 * NRHS; ++q) red[q * kBlock + tid] += red[q * kBlock + tid + w2];
          }
          __syncthreads();
        }
        if (tid == 0) {
#pragma unroll
          for (int q = 0; q < 2 * NRHS; ++q) acc[q] = red[q * kBlock];
          epi(row, acc, epi.pre(row));
        }
        __syncthreads();
      }
      ++k;
      if (k < kend) {
        cur = block_desc(a, k, CAP);
        if (cur.fits) issue(cur);
      }
    }
  }
}

// Wave-jagged engine.  Each wavefront owns one block of 64 rows; lane r
// takes the row of rank r (rows ranked by length, longest first).  At entry
// position p the rows still running are exactly ranks 0..cnt_p-1, with
// cnt_p = popcount(ballot(len > p)), and their entries sit next to each other,
// so every load instruction reads consecutive entries.  The leading entries
// of the rows of one rho-row (the H rho part, columns c N + b) share c at
// each position, so their x gathers fall on a few cache lines.  No barriers
// between the waves of a workgroup unless STAGE; kWaveUnroll positions are in
// flight per lane.  Each lane sums its row in position order, so the result
// is bitwise reproducible and independent of F32 / STAGE choices other than
// the value type.
//
// F32: read the complex64 copy of the values (wval32) instead of wval; every
// product and sum stays in double precision.
// STAGE: the rho H entries of row (a, b) gather x[a N + c] for the neighbours
// c of b, scattered over the whole rho-row a, which misses the L1 and moves a
// 128-byte line per 16-byte element.  The workgroup's four blocks (256
// consecutive rows) share a unless they straddle a rho-row, so the workgroup
// copies x[a N .. a N + N) of its first row into LDS once and every column in
// that range is read from there (any row may use it: the test is on the
// column).  Needs N * 16 bytes of dynamic LDS.
// SPLIT: phase-split values (kImagBit / kDiagBit in the column index, one
// real coefficient per entry, the diagonal from wdiag).  The complex value is
// rebuilt as (c, 0), (0, c) or the diagonal before the same fused
// multiply-adds, so every sum equals the complex layout's up to the sign of
// a zero.
// Positions in flight per lane: eight for one right-hand side, four for
// two, two for four (each position's gathers then take 4 NRHS registers).
// Launch-shape constants of the product kernels (build-time; the defaults are
// the measured best on the 1024-vertex workload): positions per gather group
// for one right-hand side (double / single-precision products), waves per
// SIMD the double and single term kernels are compiled for, and whether
// double phase-split blocks take the two-multiply-add path.  Measured per
// FP64 pass (50 intervals, 1498 products, grid 2048, four waves per SIMD):
// groups of 8 positions 104.7 ms, 6 positions 103.1, 6 with the
// two-multiply-add path 100.4, 5 positions 111.9, 4 109.2, 7 108.7; six
// positions spill at five waves.  Later (1402 products): groups of 6 at four
// waves 93.7 ms, 5 at five waves 92.1-92.3, 4 at five waves 93.3-93.4.
// Single-precision products: groups of 8 58.1 ms, 6, 12 and 16 slower.
#ifndef QSW_UNROLL1
#define QSW_UNROLL1 5
#endif
#ifndef QSW_UNROLL1_X32
#define QSW_UNROLL1_X32 8
#endif
#ifndef QSW_TERM_WAVES
#define QSW_TERM_WAVES 5
#endif
#ifndef QSW_TERM32_WAVES
#define QSW_TERM32_WAVES 4
#endif
// Waves per SIMD of term_kernel<ENGINE>: the wave layouts with double values
// QSW_TERM_WAVES; single-precision values (format 1 / 11), where five spill,
// and the CSR engines four.
// Wide groups (traversal 3: staged, double values): positions per group and
// waves per SIMD for operators with long rows.  On the complete graph of 400
// vertices (about 800 entries per row; a step to t = 10, 4008 products)
// groups of 8 at four waves took 397.7 us per product, of 7 408.6, of 6
// 419.5 and of 5 428.1, against 433 with the default five at five waves;
// ten or more spill at four waves.
#ifndef QSW_UNROLL1_WIDE
#define QSW_UNROLL1_WIDE 8
#endif
#ifndef QSW_TERM_WIDE_WAVES
#define QSW_TERM_WIDE_WAVES 4
#endif
constexpr int term_waves(int engine) {
  return engine / 100 == 3
             ? QSW_TERM_WIDE_WAVES
             : ((engine % 10 == 1 || (engine % 100 != 0 && engine % 100 != 10)) ? 4
                                                                                 : QSW_TERM_WAVES);
}
#ifndef QSW_SHARED_U1
#define QSW_SHARED_U1 8  // block-shared positions per group, one right-hand side
#endif
#ifndef QSW_FAST_NRHS
#define QSW_FAST_NRHS 2  // widest interleaved block taking the phase-split fast path
#endif
#ifndef QSW_FAST64
#define QSW_FAST64 1
#endif

// Two and four right-hand sides (estimator, batched walks): groups of 3 or 6
// (two columns) and 3 or 1 (four columns) measured level or slower.
#ifndef QSW_UNROLL2
#define QSW_UNROLL2 4
#endif
#ifndef QSW_UNROLL4
#define QSW_UNROLL4 2
#endif

#ifndef QSW_UNROLLW
#define QSW_UNROLLW 1
#endif

// single-precision values with double vectors (four waves per SIMD)
#ifndef QSW_UNROLL1_V32
#define QSW_UNROLL1_V32 6
#endif

template <int NRHS, bool X32 = false, bool F32 = false>
constexpr int wave_unroll() {
  return NRHS == 1 ? (X32 ? QSW_UNROLL1_X32 : (F32 ? QSW_UNROLL1_V32 : QSW_UNROLL1))
                   : (NRHS == 2 ? QSW_UNROLL2 : (NRHS <= 4 ? QSW_UNROLL4 : QSW_UNROLLW));
}

// A wave-uniform 64-bit value (taken from lane 0) in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Where a group of positions gathers x: anywhere (no staging, or several
// right-hand sides), global memory, the staged rho-row, global memory before
// a split position and LDS after it, or per lane through generic loads.
enum { kGatherAny = 0, kGatherGlobal, kGatherLds, kGatherSplitAt, kGatherPerLane };

// Column offset of a stored entry (column - row).
template <bool SPLIT>
__device__ __forceinline__ int64_t entry_offset(int raw) {
  if constexpr (SPLIT)
    return (int64_t)((int32_t)((uint32_t)raw << 2) >> 2);
  else
    return (int64_t)raw;
}

// v, or zero where !keep: per-component selects (a conditional expression on
// double2 itself is compiled to a branch around its operands).
__device__ __forceinline__ double2 masked(bool keep, double2 v) {
  return make_double2(keep ? v.x : 0.0, keep ? v.y : 0.0);
}
__device__ __forceinline__ float2 masked(bool keep, float2 v) {
  return make_float2(keep ? v.x : 0.0f, keep ? v.y : 0.0f);
}

// Complex value of an entry: stored (complex layouts) or rebuilt from the
// phase-split coefficient, with scalar selects only.
//
// ADJ (phase-split layouts of graph walks with a real H): the entry of
// L^dagger at the same place instead.  Off the rows (a, a), L^dagger has the
// rows of L with every Hamiltonian entry (imaginary) negated and the
// diagonal conjugated; in a row (a, a) the real off-diagonal entries of L
// are its population transfers, which L^dagger does not hold there: the
// product kernels leave the rows (a, a) to adj_diag_rows.
template <bool SPLIT, class V, class R, bool ADJ = false>
__device__ __forceinline__ V decode(int raw, R cf, V v, V dg) {
  if constexpr (!SPLIT) {
    return v;
  } else {
    const uint32_t r = (uint32_t)raw;
    const bool im = (r & kImagBit) != 0u, diag = (r & kDiagBit) != 0u;
    if constexpr (ADJ) {
      const R re = diag ? dg.x : R(0);
      const R ii = diag ? -dg.y : (im ? -cf : R(0));
      return cplxf(re, ii);
    } else {
      const R re = diag ? dg.x : (im ? R(0) : cf);
      const R ii = diag ? dg.y : (im ? cf : R(0));
      return cplxf(re, ii);
    }
  }
}

// Block k (64 rows) of the wave-jagged layout: epi(row, acc, pre) receives
// the NRHS complex sums of each row.  With STAGE, xs holds x[base ..
// base + N).  Called by a whole wavefront.
// SOA: the NRHS columns of x are consecutive n-vectors (element (c, r) at
// r n + c) instead of interleaved (c NRHS + r).  With SOA and STAGE, xs holds
// the rho-row of every column (xs[r N + i]) and `staged` says whether it
// belongs to this block's x.
// Header of block k of the wave layout, per lane: the block's first stored
// entry e0, its shared leading positions (gs, stored zero-padded to gsp at
// k wsh_stride; the lane's entry in `mine`), the position G where its rows
// enter their rho-row (-1: none, after the shared ones), the lane's row
// length after the shared positions, the longest one (rank 0), the lane's
// row (orow) and its diagonal (phase-split layouts).
struct WaveHead {
  int64_t e0;
  int gs, gsp, G, len, maxlen, orow;
  bool dfirst;  // position G holds every row's diagonal
  double2 dg;
  SharedEntry mine;  // shared entry `lane` of the block (lanes < gsp used)
};

// Stand-ins read by blocks of layouts without shared positions or G.
__device__ const SharedEntry kHeadNoShared[1] = {{0, 0u, 0.0}};
__device__ const int32_t kHeadZero32[1] = {0};
__device__ const int32_t kHeadNoG[1] = {-1};

// The header's loads, issued before any value is used (pointer selects and
// clamped lanes instead of branches) so that they cost one memory round trip
// together, and with whatever the caller issues before wave_head_use; k is
// wave-uniform.  Lanes past the block's rows read row r0 and are masked.
struct WaveRaw {
  int64_t e0;
  int n, g, len, perm;
  double2 dg;
  SharedEntry sh;
};

template <bool F32, bool SPLIT>
__device__ __forceinline__ WaveRaw wave_head_load(const SpmvArgs &a, int64_t k) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = k * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, a.n - r0);
  const int li = lane < nr ? lane : 0;
  const int64_t *pe = a.wstart ? a.wstart + k : a.rp + r0;
  const int32_t *pn = a.wshn ? a.wshn + k : kHeadZero32;
  const int32_t *pg = a.wglob ? a.wglob + k : kHeadNoG;
  // the block's shared entries sit at k wsh_stride: lane i loads entry i
  // with the header (lanes past the stride re-read the last one)
  const SharedEntry *psh = a.wshn && a.wsh_stride > 0
                               ? a.wsh + k * (int64_t)a.wsh_stride + min(lane, a.wsh_stride - 1)
                               : kHeadNoShared;
  WaveRaw w;
  w.e0 = gld(pe);
  w.n = gld(pn);
  w.g = gld(pg);
  w.sh = gld(psh);
  w.len = gld(a.wlen + r0 + li);
  w.perm = (int)gld(a.wperm + r0 + li);
  w.dg = make_double2(0.0, 0.0);
  if constexpr (SPLIT) {
    if constexpr (F32) {
      const float2 d32 = gld(a.wdiag32 + r0 + li);
      w.dg = make_double2((double)d32.x, (double)d32.y);
    } else {
      w.dg = gld(a.wdiag + r0 + li);
    }
  }
  return w;
}

__device__ __forceinline__ WaveHead wave_head_use(const SpmvArgs &a, int64_t k, const WaveRaw &w) {
  const int lane = threadIdx.x & 63;
  const int nr = (int)min((int64_t)kWaveRows, a.n - k * kWaveRows);
  WaveHead h;
  h.e0 = uniform64(w.e0);
  h.gs = __builtin_amdgcn_readfirstlane(w.n);
  h.gsp = (h.gs + kSharedPad - 1) / kSharedPad * kSharedPad;  // zero-padded count
  h.mine = w.sh;
  const int g = __builtin_amdgcn_readfirstlane(w.g);
  h.G = g >= 0 ? (g & kGlobMask) - h.gs : -1;
  h.dfirst = g >= 0 && (g & kGlobDiagFirst) != 0;
  h.len = lane < nr ? w.len - h.gs : 0;
  h.maxlen = __builtin_amdgcn_readfirstlane(h.len);
  h.orow = lane < nr ? w.perm : 0;
  h.dg = w.dg;
  return h;
}

template <bool F32, bool SPLIT>
__device__ __forceinline__ WaveHead wave_head(const SpmvArgs &a, int64_t k) {
  return wave_head_use(a, k, wave_head_load<F32, SPLIT>(a, k));
}

template <int NRHS, bool F32, bool STAGE, class Epi, bool SOA = false, bool SPLIT = false,
          bool X32 = false, bool ADJ = false, int UNR = 0>
__device__ __forceinline__ void wave_block_h(const SpmvArgs &a, int64_t k, const WaveHead &hd,
                                             Epi &epi, const VecT<X32> *xs, int64_t base,
                                             bool staged = true, int64_t span = 0) {
  // X32: complex64 x, single-precision values and sums (F32 layouts only)
  static_assert(!X32 || F32, "single-precision products read single-precision values");
  // ADJ: products with L^dagger through the layout of L (see decode)
  static_assert(!ADJ || (SPLIT && !X32 && !SOA), "adjoint products read phase-split double layouts");
  using V = VecT<X32>;
  using R = RealT<X32>;
  // one right-hand side: xs holds x[base .. base + span) (span = N by default)
  const uint64_t lim = (uint64_t)(span ? span : a.N);
  // positions per group (UNR: the caller's, else the default for the types)
  constexpr int kWaveUnroll = UNR > 0 ? UNR : wave_unroll<NRHS, X32, F32>();
  const int lane = threadIdx.x & 63;
  const int64_t r0 = k * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, a.n - r0);
  const int64_t e0 = hd.e0;
  const int gsp = hd.gsp;
  const int len = hd.len;
  const int maxlen = hd.maxlen;
  const int orow = hd.orow;
  typename Epi::Pre pre{};
  if (lane < nr) pre = epi.pre(r0 + orow);
  // ADJ: rows (a, a) are left to adj_diag_rows
  bool adj_skip = false;
  if constexpr (ADJ) {
    const int64_t row = r0 + orow;
    adj_skip = row == (row / a.N) * ((int64_t)a.N + 1);
  }
  const V dg = cplx<V>(hd.dg.x, hd.dg.y);  // exact: single values come from floats
  R acc[2 * NRHS];
#pragma unroll
  for (int q = 0; q < 2 * NRHS; ++q) acc[q] = R(0);
  // Shared leading positions: one entry for the whole block (the same for
  // every lane's row), gathering x at row + off from global memory.  They come
  // first in every row, as in the per-row order, and the zero padding adds
  // nothing, so the sums are those of the unshared layout.
  if (gsp > 0) {
    const int64_t row = r0 + orow;
    constexpr int SU = NRHS == 1 ? QSW_SHARED_U1
                                 : (NRHS == 2 ? kSharedPad / 2 : (NRHS <= 4 ? kSharedPad / 4 : 1));
    static_assert(kSharedPad % SU == 0, "shared groups divide the padding");
    // lane i loaded entry i with the block header (at most kSharedMax
    // entries), and each group takes its entries from the lanes (no load
    // between the groups' gathers)
    static_assert(kSharedMax <= 64, "one shared entry per lane");
    {
      const int cnt = gsp;  // a multiple of SU
      const SharedEntry mine = hd.mine;
      const unsigned long long mine_coef = (unsigned long long)__double_as_longlong(mine.coef);
      // one group of S positions: S gathers in flight, then the sums (wider
      // groups of 16 measured no faster)
      // A shared entry is real or imaginary (c or i c, phase-split values):
      // for one or two right-hand sides its product takes the two
      // multiply-adds of the complex product that do not multiply by zero, in
      // the same order, chosen by a wave-uniform branch, so the sums are
      // those of the complex product up to the sign of a zero (FP64 pass
      // 92.5 -> 91.9 ms, single-precision products 44.7 -> 44.2 ms); four
      // (the batch engine) keep the complex product, whose registers the
      // branch would spill.
      auto sgroup = [&](auto width, int p) {
        constexpr int S = decltype(width)::value;
        R cm[S];
        bool imu[S];
        int64_t c[S];
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const int off = __builtin_amdgcn_readlane(mine.off, p + u);
          const uint32_t flags = (uint32_t)__builtin_amdgcn_readlane((int)mine.flags, p + u);
          const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine_coef, p + u);
          const uint32_t hi =
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine_coef >> 32), p + u);
          const double e = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
          const R cf = F32 ? (R)(float)e : (R)e;
          imu[u] = (flags & kImagBit) != 0u;
          // wave-uniform (lanes past the block's rows gather at row r0, in
          // bounds, and their sums are never written); ADJ: a shared real
          // entry is a population transfer of a lone row (a, a) (decode)
          cm[u] = ADJ ? (imu[u] ? -cf : R(0)) : cf;
          c[u] = row + off;
        }
        V xg[S][NRHS];
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
          for (int r = 0; r < NRHS; ++r)
            xg[u][r] = gld(xbase<X32>(a) + (SOA ? (int64_t)r * a.n + c[u] : c[u] * NRHS + r));
#pragma unroll
        for (int u = 0; u < S; ++u) {
          if constexpr (NRHS <= 2) {
            if (imu[u]) {
#pragma unroll
              for (int r = 0; r < NRHS; ++r) {
                acc[2 * r] = rfma(-cm[u], xg[u][r].y, acc[2 * r]);
                acc[2 * r + 1] = rfma(cm[u], xg[u][r].x, acc[2 * r + 1]);
              }
            } else {
#pragma unroll
              for (int r = 0; r < NRHS; ++r) {
                acc[2 * r] = rfma(cm[u], xg[u][r].x, acc[2 * r]);
                acc[2 * r + 1] = rfma(cm[u], xg[u][r].y, acc[2 * r + 1]);
              }
            }
          } else {
            const V v = imu[u] ? cplxf(R(0), cm[u]) : cplxf(ADJ ? R(0) : cm[u], R(0));
#pragma unroll
            for (int r = 0; r < NRHS; ++r) cmac(acc[2 * r], acc[2 * r + 1], v, xg[u][r]);
          }
        }
      };
      for (int p = 0; p < cnt; p += SU) sgroup(std::integral_constant<int, SU>{}, p);
    }
  }
  // Branch-free groups of kWaveUnroll positions.  Position p's entries start
  // at the wave-uniform offset ps_p, so lane l reads entry e0 + ps_p + l
  // whether or not its row is still running (entries past the row belong to
  // other rows, the next block or the zero padding after the arrays: always
  // in bounds) and discards the product when it is not, gathering x at its
  // own row then.  With no branch around them, every load of a group is
  // issued before the first wait.
  const int32_t *cb = a.wcol + e0;
  const int64_t lane_row = r0 + orow;
  int ps = 0;
  int gsplit = 0;
  // one group: column indices and values, then the x gathers (MODE), then
  // the multiply-adds in position order
  auto group = [&](auto mode, int p0) {
    constexpr int MODE = decltype(mode)::value;
    int bcur[kWaveUnroll];
    bool ok[kWaveUnroll];
#pragma unroll
    for (int u = 0; u < kWaveUnroll; ++u) {
      const int cnt = __popcll(__ballot(len > p0 + u));
      ok[u] = lane < cnt;
      bcur[u] = ps + lane;
      ps += cnt;
    }
    int c[kWaveUnroll];
#pragma unroll
    for (int u = 0; u < kWaveUnroll; ++u) c[u] = load_entry(cb + bcur[u]);
    V v[kWaveUnroll];
    R cf[kWaveUnroll];
#pragma unroll
    for (int u = 0; u < kWaveUnroll; ++u) {
      if constexpr (SPLIT) {
        if constexpr (X32)
          cf[u] = gld(a.wcoef32 + e0 + bcur[u]);
        else
          cf[u] = F32 ? load_entry(a.wcoef32 + e0 + bcur[u]) : load_entry(a.wcoef + e0 + bcur[u]);
        v[u] = dg;  // unused
      } else {
        if constexpr (X32)
          v[u] = gld(a.wval32 + e0 + bcur[u]);
        else
          v[u] = F32 ? load_entry(a.wval32 + e0 + bcur[u]) : load_entry(a.wval + e0 + bcur[u]);
        cf[u] = R(0);  // unused
      }
    }
    // a lane past its row's end read another row's entry: its offset is
    // relative to that row, so the lane gathers at its own row instead
    int64_t col[kWaveUnroll];
#pragma unroll
    for (int u = 0; u < kWaveUnroll; ++u)
      col[u] = lane_row + (ok[u] ? entry_offset<SPLIT>(c[u]) : 0);
    if constexpr (MODE == kGatherAny) {
      // no staging: global gathers first (they need the columns only), the
      // values decoded where they are used
      V xg[kWaveUnroll][NRHS];
#pragma unroll
      for (int u = 0; u < kWaveUnroll; ++u)
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
          xg[u][r] = gld(xbase<X32>(a) + (SOA ? (int64_t)r * a.n + col[u] : col[u] * NRHS + r));
#pragma unroll
      for (int u = 0; u < kWaveUnroll; ++u) {
        const V vz = masked(ok[u], decode<SPLIT, V, R, ADJ>(c[u], cf[u], v[u], dg));
#pragma unroll
        for (int r = 0; r < NRHS; ++r) cmac(acc[2 * r], acc[2 * r + 1], vz, xg[u][r]);
      }
    } else {
      // staged: xs holds the staged rho-row of every column (xs[r N' + o],
      // N' = lim for one column); column r of x at r n + col (SOA) or col
      V xv[kWaveUnroll][NRHS];
#pragma unroll
      for (int u = 0; u < kWaveUnroll; ++u) {
        const uint64_t o = (uint64_t)((int64_t)col[u] - base);
        const uint64_t oc = o < lim ? o : 0;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) {
          // column r: SOA at r n + col (staged at r lim + o), else
          // interleaved at col NRHS + r (staged at o NRHS + r)
          const V *xgp = SOA ? xbase<X32>(a) + (int64_t)r * a.n + col[u] : xbase<X32>(a) + col[u] * NRHS + r;
          const V *xlp = SOA ? xs + (uint64_t)r * lim : xs + r;
          constexpr uint64_t ls = SOA ? 1 : NRHS;  // LDS stride between rho-row elements
          if constexpr (MODE == kGatherGlobal)
            xv[u][r] = gld(xgp);
          else if constexpr (MODE == kGatherLds)
            xv[u][r] = xlp[oc * ls];
          else if constexpr (MODE == kGatherSplitAt)  // before `gsplit` global, then LDS
            xv[u][r] = *(p0 + u < gsplit ? xgp : xlp + oc * ls);
          else  // kGatherPerLane
            xv[u][r] = *(o < lim ? xlp + o * ls : xgp);
        }
      }
#pragma unroll
      for (int u = 0; u < kWaveUnroll; ++u) {
        const V vz = masked(ok[u], decode<SPLIT, V, R, ADJ>(c[u], cf[u], v[u], dg));
#pragma unroll
        for (int r = 0; r < NRHS; ++r) cmac(acc[2 * r], acc[2 * r + 1], vz, xv[u][r]);
      }
    }
  };
  // Phase-split fast path (one or two interleaved right-hand sides): in a
  // regular block whose position G holds every row's diagonal, every other
  // entry is real or
  // imaginary, and such an entry's product takes two multiply-adds with the
  // components of x chosen by its phase; they are the complex product's
  // multiply-adds that do not multiply by zero, in the same order, so the
  // sums are the generic path's up to the sign of a zero.  The diagonal at G
  // is a full complex product with x at the lane's own row.  Offsets into the
  // staged rho-row are 32-bit.  Taken for single-precision values: on the
  // 1024-vertex operator it measured 81.5 -> 80.0 us per Taylor-term product
  // there, but 77.6 -> 78.7 us with double values (whose product kernel is
  // at the edge of its register budget).
  bool fast = false;
  if constexpr (STAGE && SPLIT && (F32 || QSW_FAST64) && NRHS <= QSW_FAST_NRHS && !SOA) {
    const int G = hd.G;
    const int64_t rho = r0 / a.N * a.N;
    if (G >= 0 && hd.dfirst && (uint64_t)(rho - base) < lim) {
      fast = true;
      const int lrel = (int)(lane_row - base);  // the lane's row in the staged rows
      const uint32_t lmax = (uint32_t)lim - 1u;
      // positions p0 .. min(p0 + kWaveUnroll, pend) - 1, gathering from
      // global memory (MODE kGatherGlobal) or the staged rows (kGatherLds);
      // column r of x at row NRHS + r in both
      auto fgroup = [&](auto mode, int p0, int pend) {
        constexpr int MODE = decltype(mode)::value;
        int bcur[kWaveUnroll];
        bool ok[kWaveUnroll];
#pragma unroll
        for (int u = 0; u < kWaveUnroll; ++u) {
          const int cnt = p0 + u < pend ? __popcll(__ballot(len > p0 + u)) : 0;
          ok[u] = lane < cnt;
          bcur[u] = ps + lane;
          ps += cnt;
        }
        int c[kWaveUnroll];
        R cf[kWaveUnroll];
#pragma unroll
        for (int u = 0; u < kWaveUnroll; ++u) c[u] = load_entry(cb + bcur[u]);
#pragma unroll
        for (int u = 0; u < kWaveUnroll; ++u) {
          if constexpr (X32)
            cf[u] = gld(a.wcoef32 + e0 + bcur[u]);
          else
            cf[u] = F32 ? load_entry(a.wcoef32 + e0 + bcur[u]) : load_entry(a.wcoef + e0 + bcur[u]);
        }
        V xv[kWaveUnroll][NRHS];
#pragma unroll
        for (int u = 0; u < kWaveUnroll; ++u) {
          const int off = ok[u] ? (int)((uint32_t)c[u] << 2) >> 2 : 0;
#pragma unroll
          for (int r = 0; r < NRHS; ++r) {
            if constexpr (MODE == kGatherLds)
              xv[u][r] = xs[min((uint32_t)(lrel + off), lmax) * NRHS + r];
            else
              xv[u][r] = gld(xbase<X32>(a) + (lane_row + off) * NRHS + r);
          }
        }
#pragma unroll
        for (int u = 0; u < kWaveUnroll; ++u) {
          const bool im = ((uint32_t)c[u] & kImagBit) != 0u;
          // ADJ: Hamiltonian entries negated, real ones (transfers) dropped
          const R cm = ok[u] ? (ADJ ? (im ? -cf[u] : R(0)) : cf[u]) : R(0);
#pragma unroll
          for (int r = 0; r < NRHS; ++r) {
            const R sx = im ? xv[u][r].y : xv[u][r].x;
            const R sy = im ? xv[u][r].x : xv[u][r].y;
            acc[2 * r] = rfma(im ? -cm : cm, sx, acc[2 * r]);
            acc[2 * r + 1] = rfma(cm, sy, acc[2 * r + 1]);
          }
        }
      };
      int p0 = 0;
      for (; p0 < G; p0 += kWaveUnroll) fgroup(std::integral_constant<int, kGatherGlobal>{}, p0, G);
      {
        // position G: every running row's diagonal (stored in the stream as
        // a marker, its value in dg)
        const int cnt = __popcll(__ballot(len > G));
        const V vz = masked(lane < cnt, ADJ ? cplxf(dg.x, -dg.y) : dg);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) cmac(acc[2 * r], acc[2 * r + 1], vz, xs[lrel * NRHS + r]);
        ps += cnt;
      }
      for (p0 = G + 1; p0 < maxlen; p0 += kWaveUnroll)
        fgroup(std::integral_constant<int, kGatherLds>{}, p0, maxlen);
    }
  }
  if (fast) {
    // done above
  } else if constexpr (STAGE) {
    // The layout puts each row's entries outside its rho-row first; in a
    // block whose rows share one rho-row and all leave it at the same
    // position G (wglob[k] = G, else -1), positions < G gather from global
    // memory and the rest from the staged rho-row.  Other blocks choose per
    // lane with generic loads, and blocks whose rho-row is not staged (SOA:
    // `staged` false) gather from global memory throughout.
    const int G = hd.G;
    const int64_t rho = r0 / a.N * a.N;
    const bool regular = G >= 0 && (uint64_t)(rho - base) < lim;
    int p0 = 0;
    if (SOA && !staged) {
      for (; p0 < maxlen; p0 += kWaveUnroll)
        group(std::integral_constant<int, kGatherGlobal>{}, p0);
    } else if (regular) {
      const int gend = min(G, maxlen);
      for (; p0 + kWaveUnroll <= gend; p0 += kWaveUnroll)
        group(std::integral_constant<int, kGatherGlobal>{}, p0);
      if (p0 < gend) {
        gsplit = gend;
        group(std::integral_constant<int, kGatherSplitAt>{}, p0);
        p0 += kWaveUnroll;
      }
      for (; p0 < maxlen; p0 += kWaveUnroll) group(std::integral_constant<int, kGatherLds>{}, p0);
    } else {
      for (; p0 < maxlen; p0 += kWaveUnroll)
        group(std::integral_constant<int, kGatherPerLane>{}, p0);
    }
  } else {
    for (int p0 = 0; p0 < maxlen; p0 += kWaveUnroll)
      group(std::integral_constant<int, kGatherAny>{}, p0);
  }
  if (lane < nr && !adj_skip) epi(r0 + orow, acc, pre);
}

template <int NRHS, bool F32, bool STAGE, class Epi, bool SOA = false, bool SPLIT = false,
          bool X32 = false>
__device__ __forceinline__ void wave_block(const SpmvArgs &a, int64_t k, Epi &epi,
                                           const VecT<X32> *xs, int64_t base, bool staged = true,
                                           int64_t span = 0) {
  const WaveHead hd = wave_head<F32, SPLIT>(a, k);
  wave_block_h<NRHS, F32, STAGE, Epi, SOA, SPLIT, X32>(a, k, hd, epi, xs, base, staged, span);
}

// xs[0 .. cnt) = src[0 .. cnt) by the whole workgroup, cnt at most the
// staging budget (kStageMaxBytes): straight-line code with every load issued
// before the first LDS write (a load-wait-write loop takes one memory round
// trip per kBlock elements, and a loop head makes the compiler wait for the
// loads issued before it).  The guards are wave-uniform.
constexpr int kStageMaxPerThread = (int)((kStageMaxBytes / sizeof(double2) + kBlock - 1) / kBlock);

template <class T>
__device__ __forceinline__ void stage_copy(T *xs, const T *src, int cnt) {
  T v[kStageMaxPerThread];
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kStageMaxPerThread; ++u)
    if (u * kBlock < cnt) v[u] = gld(src + min(t + u * kBlock, cnt - 1));
#pragma unroll
  for (int u = 0; u < kStageMaxPerThread; ++u)
    if (u * kBlock < cnt && t + u * kBlock < cnt) xs[t + u * kBlock] = v[u];
}

// `grid`: the workgroups that take blocks (0: all of the launch).
template <int NRHS, bool F32, bool STAGE, bool SPLIT, class Epi, bool X32 = false,
          bool ADJ = false, int UNR = 0>
__device__ __forceinline__ void wave_engine(const SpmvArgs &a, Epi &epi, int grid = 0) {
  constexpr int WPB = kBlock / 64;  // wavefronts per workgroup
  const int64_t nw = (int64_t)(grid > 0 ? grid : (int)gridDim.x) * WPB;
  extern __shared__ double2 xs_lds[];
  VecT<X32> *xs = reinterpret_cast<VecT<X32> *>(xs_lds);
  for (int64_t kb = (int64_t)blockIdx.x * WPB; kb < a.nwb; kb += nw) {
    const int64_t k = kb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // the block header's loads are issued before the staging (a wave past
    // the last block reads the last one's and does nothing with it), so the
    // two share one memory round trip
    const WaveRaw raw = wave_head_load<F32, SPLIT>(a, k < a.nwb ? k : a.nwb - 1);
    int64_t base = 0;
    if constexpr (STAGE) {
      // rho-row of the workgroup's first row, all NRHS interleaved columns
      base = (kb * kWaveRows) / a.N * a.N;
      if (kb != (int64_t)blockIdx.x * WPB) __syncthreads();  // the previous blocks are done with xs
      stage_copy(xs, xbase<X32>(a) + base * NRHS, a.N * NRHS);
      __syncthreads();
    }
    if (k < a.nwb)
      wave_block_h<NRHS, F32, STAGE, Epi, false, SPLIT, X32, ADJ, UNR>(
          a, k, wave_head_use(a, k, raw), epi, xs, base);
  }
}

// XCD-banded traversal (engines 200 / 201, N = 512, 1024 or 2048).  The
// dispatcher deals workgroups to the 8 XCDs in turn, so workgroup w runs on
// XCD w mod 8.  XCD x takes the rows (a, b) whose b lies in its band of N/8
// columns, for every a: the H rho gathers x[c N + b] then stay within the
// band's N x N/8 slice of x, which fits the XCD's L2, instead of ranging
// over all of x.  A workgroup takes four consecutive blocks of its band;
// they span 4/bw rho-rows (bw = band blocks per rho-row), whose x rows are
// staged in LDS for the rho H gathers.  Only the order of the blocks
// changes: every row's sum is the same as in the other engines.
__device__ __forceinline__ int band_blocks(int N) { return N / 64 / 8; }
__device__ __forceinline__ int band_rows(int N) {
  const int bw = band_blocks(N);
  return bw >= 4 ? 1 : 4 / bw;
}

template <bool F32, bool SPLIT, class Epi>
__device__ __forceinline__ void wave_engine_banded(const SpmvArgs &a, Epi &epi) {
  constexpr int WPB = kBlock / 64;
  // a workgroup takes four blocks of its band: other workgroup sizes build
  // without this traversal (banded_ok is false for them)
  if constexpr (WPB != 4) return;
  extern __shared__ double2 xs[];
  const int64_t nbr = a.N / 64;         // blocks per rho-row
  const int64_t bw = band_blocks(a.N);  // band blocks per rho-row
  const int64_t rows = band_rows(a.N);
  const int xcd = blockIdx.x & 7;
  const int64_t wi = blockIdx.x >> 3, g8 = gridDim.x >> 3;
  const int64_t nq = (int64_t)a.N * bw / WPB;  // quads per band
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int64_t q = wi; q < nq; q += g8) {
    const int64_t i0 = q * WPB;
    const int64_t base = (i0 / bw) * a.N;
    const int64_t bi = i0 + wave;
    const int64_t k = (bi / bw) * nbr + xcd * bw + bi % bw;
    // header loads before the staging, as in wave_engine
    const WaveRaw raw = wave_head_load<F32, SPLIT>(a, k);
    if (q != wi) __syncthreads();  // the previous quad is done with xs
    stage_copy(xs, a.x + base, (int)(rows * a.N));
    __syncthreads();
    wave_block_h<1, F32, true, Epi, false, SPLIT>(a, k, wave_head_use(a, k, raw), epi, xs, base,
                                                  true, rows * a.N);
  }
}

template <int LPR, class Epi>
__device__ __forceinline__ void vector_engine(const SpmvArgs &a, Epi &epi) {
  constexpr int RPI = kBlock / LPR;
  const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t r1 = min(a.n, r0 + a.rows_per_block);
  for (int64_t base = r0; base < r1; base += RPI) {
    const int64_t row = base + g;
    double acc[2] = {0.0, 0.0};
    if (row < r1) {
      for (int64_t e = a.rp[row] + lane; e < a.rp[row + 1]; e += LPR)
        cmac(acc[0], acc[1], load_csr(a.val + e), a.x[load_csr(a.col + e)]);
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      acc[0] += __shfl_xor(acc[0], off, LPR);
      acc[1] += __shfl_xor(acc[1], off, LPR);
    }
    if (row < r1 && lane == 0) epi(row, acc, epi.pre(row));
  }
}

// Engines: wave-jagged traversal 0 (plain), 100 (rho-row staged in LDS), 200
// (staged and XCD-banded) or 300 (staged, wide groups at four waves per
// SIMD, double values only), plus 1 for single-precision values and 10 for
// phase-split values; 3 = CSR stream, 4..64 = vector with that many lanes per
// row.
template <int ENGINE>
constexpr bool is_vector_engine() {
  return ENGINE == 4 || ENGINE == 8 || ENGINE == 16 || ENGINE == 32 || ENGINE == 64;
}

template <int ENGINE, class Epi>
__device__ __forceinline__ void run_engine(const SpmvArgs &a, Epi &epi) {
  if constexpr (ENGINE == 3) {
    stream_engine<1>(a, epi);
  } else if constexpr (is_vector_engine<ENGINE>()) {
    vector_engine<ENGINE>(a, epi);
  } else {
    constexpr int trav = ENGINE / 100, fmt = ENGINE % 100;
    static_assert(trav <= 3 && (fmt == 0 || fmt == 1 || fmt == 10 || fmt == 11), "engine");
    static_assert(trav != 3 || fmt % 10 == 0, "wide groups: double values");
    constexpr bool f32 = (fmt % 10) == 1, split = fmt >= 10;
    if constexpr (trav == 2)
      wave_engine_banded<f32, split>(a, epi);
    else if constexpr (trav == 3)
      wave_engine<1, f32, true, split, Epi, false, false, QSW_UNROLL1_WIDE>(a, epi);
    else
      wave_engine<1, f32, trav == 1, split>(a, epi);
  }
}

// ---------------------------------------------------------------- epilogues

// Each epilogue names what it reads per row (Pre) so the engine can fetch it
// ahead of the reduction.
struct NoPre {};

struct TaylorEpi {  // y = alpha A x ; F_out = F_in + y ; norms
  const SpmvArgs &a;
  unsigned long long mb = 0, mf = 0, mb0 = 0;
  typedef double2 Pre;
  __device__ explicit TaylorEpi(const SpmvArgs &args) : a(args) {}
  __device__ __forceinline__ Pre pre(int64_t row) const { return a.fin[row]; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre f) {
    const double2 y = make_double2(a.alpha * acc[0], a.alpha * acc[1]);
    a.y[row] = y;
    if (a.j == 1) mb0 = umax(mb0, abs_bits(cabs2(f)));
    f.x += y.x;
    f.y += y.y;
    a.fout[row] = f;
    mb = umax(mb, abs_bits(cabs2(y)));
    mf = umax(mf, abs_bits(cabs2(f)));
  }
};

struct PlainEpi {  // y = alpha A x
  const SpmvArgs &a;
  typedef NoPre Pre;
  __device__ explicit PlainEpi(const SpmvArgs &args) : a(args) {}
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre) {
    a.y[row] = make_double2(a.alpha * acc[0], a.alpha * acc[1]);
  }
};

struct PowerEpi {  // y = alpha A x ; max |y|
  const SpmvArgs &a;
  unsigned long long mk = 0;
  typedef NoPre Pre;
  __device__ explicit PowerEpi(const SpmvArgs &args) : a(args) {}
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre) {
    const double2 y = make_double2(a.alpha * acc[0], a.alpha * acc[1]);
    a.y[row] = y;
    mk = umax(mk, abs_bits(cabs2(y)));
  }
};

struct Spmm2Epi {  // two right-hand sides for the 1-norm estimator
  double2 *Y;
  int mode;
  double2 *sgn;
  double *h;
  double s0 = 0.0, s1 = 0.0;
  typedef NoPre Pre;
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre) {
    const double2 y0 = make_double2(acc[0], acc[1]), y1 = make_double2(acc[2], acc[3]);
    Y[2 * row] = y0;
    Y[2 * row + 1] = y1;
    const double m0 = cabs2(y0), m1 = cabs2(y1);
    if (mode == 1) {
      s0 += m0;
      s1 += m1;
      sgn[2 * row] = m0 > 0.0 ? make_double2(y0.x / m0, y0.y / m0) : make_double2(1.0, 0.0);
      sgn[2 * row + 1] = m1 > 0.0 ? make_double2(y1.x / m1, y1.y / m1) : make_double2(1.0, 0.0);
    } else if (mode == 2) {
      h[row] = m0 > m1 ? m0 : m1;
    }
  }
};

// --------------------------------------------------------------------------
// Superoperator assembly: one wavefront per 64-row block (grid-stride over
// blocks).  Lane i first loads row r0 + i's descriptors (all rows' loads in
// one round trip); then the rows are written one after the other, the lanes
// covering consecutive entries of a row, so that every column and value
// store of the wave is contiguous.
// --------------------------------------------------------------------------
struct AsmRow {
  int64_t start, ha0, hb0, ra0;
  int32_t d0, r1, len;  // H rho entries, + diagonal + rho H entries, all entries
  int32_t a, b;
  double2 dval;
};

__device__ __forceinline__ AsmRow asm_row(const AssembleArgs &A, int64_t r) {
  const int64_t N = A.N;
  const double ch = A.sigma * (1.0 - A.omega);  // sigma (1 - omega)
  const double w = A.rscale;                    // omega, or 1 for pre-scaled rates
  const int64_t a = r / N, b = r - a * N;
  const int64_t ha0 = A.hp[a], ha1 = A.hp[a + 1];
  const int64_t hb0 = A.hp[b], hb1 = A.hp[b + 1];
  const int64_t ra0 = A.rp[a], ra1 = A.rp[a + 1];
  const int64_t degHa = ha1 - ha0, degHb = hb1 - hb0, degRa = ra1 - ra0;
  AsmRow R;
  // Rows before (a, 0): sum over a' < a of (N degH(a') + E_H + N + degR(a'));
  // rows (a, b') with b' < b: b' (degH(a) + 1) + degH(b') plus the
  // population-transfer entries of row (a, a) once b > a.
  R.start = N * A.PH[a] + a * (A.EH + N) + A.PR[a] + b * (degHa + 1) + A.PH[b] +
            (b > a ? degRa : 0);
  R.ha0 = ha0;
  R.hb0 = hb0;
  R.ra0 = ra0;
  R.d0 = (int32_t)degHa;
  R.r1 = (int32_t)(degHa + 1 + degHb);
  R.len = R.r1 + (int32_t)(a == b ? degRa : 0);
  R.a = (int32_t)a;
  R.b = (int32_t)b;
  // diagonal: sigma(-i)(1-w)(H_aa - H_bb) - w/2 (K_a + K_b) + [a==b] w R_aa
  R.dval = make_double2(-0.5 * w * (A.K[a] + A.K[b]) + (a == b ? w * A.rdiag[a] : 0.0),
                        -ch * (A.hdiag[a] - A.hdiag[b]));
  return R;
}

__device__ __forceinline__ int64_t rd64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double rdd(double v, int l) {
  return __longlong_as_double(rd64(__double_as_longlong(v), l));
}

__global__ __launch_bounds__(kBlock) void assemble_kernel(AssembleArgs A, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
  const int64_t N = A.N;
  const double ch = A.sigma * (1.0 - A.omega);
  const double w = A.rscale;
  for (int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); k < nwb;
       k += nwaves) {
    const int64_t r0 = k * kWaveRows;
    const int nr = (int)min((int64_t)kWaveRows, n - r0);
    const AsmRow mine = asm_row(A, r0 + (lane < nr ? lane : 0));
    if (lane < nr) A.row_ptr[r0 + lane] = mine.start;
    if (r0 + nr == n && lane == 0) A.row_ptr[n] = 2 * N * A.EH + N * N + A.PR[N];
    for (int i = 0; i < nr; ++i) {
      // row r0 + i, from lane i (wave-uniform)
      const int64_t start = rd64(mine.start, i);
      const int64_t ha0 = rd64(mine.ha0, i), hb0 = rd64(mine.hb0, i), ra0 = rd64(mine.ra0, i);
      const int d0 = __builtin_amdgcn_readlane(mine.d0, i);
      const int r1 = __builtin_amdgcn_readlane(mine.r1, i);
      const int len = __builtin_amdgcn_readlane(mine.len, i);
      const int64_t a = __builtin_amdgcn_readlane(mine.a, i);
      const int64_t b = __builtin_amdgcn_readlane(mine.b, i);
      const double2 dval = make_double2(rdd(mine.dval.x, i), rdd(mine.dval.y, i));
      // Each row in structural order: the H rho entries (column c N + b,
      // ascending c), the diagonal, the rho H entries (column a N + c,
      // ascending c), then the population-transfer entries (column
      // j (N + 1), ascending j).  Rows of one rho-row a then share the
      // column offsets c N of their leading entries, which the product
      // kernels use to coalesce gathers.
      for (int e = lane; e < len; e += 64) {
        int32_t c;
        double2 v;
        if (e < d0) {  // sigma(-i)(1-w) H_ac on rho_cb
          const double2 h = A.hv[ha0 + e];
          c = (int32_t)((int64_t)A.hc[ha0 + e] * N + b);
          v = make_double2(ch * h.y, -ch * h.x);
        } else if (e == d0) {
          c = (int32_t)(a * N + b);
          v = dval;
        } else if (e < r1) {  // sigma(+i)(1-w) conj(H_bc) on rho_ac
          const int64_t j = hb0 + (e - d0 - 1);
          const double2 h = A.hv[j];
          c = (int32_t)(a * N + A.hc[j]);
          v = make_double2(ch * h.y, ch * h.x);
        } else {  // w R_aj on rho_jj
          const int64_t j = ra0 + (e - r1);
          c = (int32_t)((int64_t)A.rc[j] * (N + 1));
          v = make_double2(w * A.rv[j], 0.0);
        }
        A.col[start + e] = c;
        A.val[start + e] = v;
      }
    }
  }
}

// Row blocks of the stream engine: block k starts at the first row whose
// first entry index is >= k B.
__global__ void row_blocks_kernel(const int64_t *rp, int64_t n, int64_t B, int32_t *blk,
                                  int64_t nblk) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nblk) return;
  if (k == nblk) {
    blk[k] = (int32_t)n;
    return;
  }
  const int64_t target = k * B;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  blk[k] = (int32_t)lo;
}

// Wave-jagged layout of a CSR, one wavefront per 64-row block: rank the
// rows by length (longest first, ties by row), then scatter the entries
// position-major (entry p of rank r at the block's start + entries of
// positions < p + r).  Inside each row the entries outside the row's own
// rho-row (columns c N + b of the H rho part, population transfer) come first
// and those inside it (the rho H part and the diagonal) last, each group in
// column order: all rows of a block share their rho-row, so every position of
// the block gathers from global memory for all rows or from the staged
// rho-row for all rows.  Leading positions whose entry has the same offset
// from its row and the same value in every row of the block are stored once
// for the block (SharedEntry) when phase-split values are built.

// Row of lane `lane` in its block: CSR start, length (-1 for lanes past the
// last row), the number of its entries outside its rho-row and, when its
// entries inside the rho-row are consecutive in the CSR (as the assembled
// rows are: H rho part, diagonal and rho H part, population transfer), the
// range [lo, hi) they occupy.
struct WjagRow {
  int64_t row, src0;
  int len, outside;
  int lo, hi;
  bool consecutive;
  int64_t rho0;  // first column of the row's rho-row
  int32_t N;
  __device__ bool inside(const int32_t *col, int i) const {
    return (uint64_t)((int64_t)col[src0 + i] - rho0) < (uint64_t)N;
  }
};

__device__ __forceinline__ WjagRow wjag_row(const int64_t *rp, const int32_t *col, int64_t r0,
                                            int nr, int32_t N, int lane) {
  WjagRow w;
  w.row = r0 + lane;
  w.src0 = lane < nr ? rp[w.row] : 0;
  w.len = lane < nr ? (int)(rp[w.row + 1] - w.src0) : -1;
  w.N = N;
  w.rho0 = w.row / N * N;
  int first = -1, last = -1, in = 0;
  // eight column loads in flight per step (clamped into the row, so a row
  // shorter than the step re-reads its last entry)
  for (int i0 = 0; i0 < w.len; i0 += 8) {
    int32_t c8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c8[u] = col[w.src0 + min(i0 + u, w.len - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u;
      if (i < w.len && (uint64_t)((int64_t)c8[u] - w.rho0) < (uint64_t)N) {
        if (first < 0) first = i;
        last = i;
        ++in;
      }
    }
  }
  w.outside = w.len < 0 ? 0 : w.len - in;
  w.consecutive = in == 0 || last - first + 1 == in;
  w.lo = in ? first : max(w.len, 0);
  w.hi = in ? last + 1 : max(w.len, 0);
  return w;
}

// CSR index of entry q (outside-first order) of a row whose inside entries
// are consecutive: position arithmetic.
__device__ __forceinline__ int64_t wjag_consecutive_index(const WjagRow &w, int q) {
  const int tail = w.len - w.hi;  // outside entries after the inside ones
  if (q < w.lo) return w.src0 + q;
  if (q < w.lo + tail) return w.src0 + w.hi + (q - w.lo);
  return w.src0 + w.lo + (q - w.lo - tail);
}

// Loads of entries q0 .. q0 + 7 of the lane's row (consecutive rows only),
// issued together; positions past the row re-read its last entry, and a lane
// without entries reads entry 0 of the CSR (callers have nnz > 0).
__device__ __forceinline__ void wjag_load8(const int32_t *col, const double2 *val, const WjagRow &w,
                                           int q0, int32_t (&cc)[8], double2 (&vv)[8]) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t e = w.len > 0 ? wjag_consecutive_index(w, min(q0 + u, w.len - 1)) : 0;
    cc[u] = col[e];
    vv[u] = val[e];
  }
}

// CSR index of the row's entry q in the outside-first order: by position
// arithmetic when the inside entries are consecutive, else with the cursors
// io, ii over the outside and inside entries (advanced in order of q).
__device__ __forceinline__ int64_t wjag_next(const int32_t *col, const WjagRow &w, int q, int &io,
                                             int &ii) {
  if (w.consecutive) return wjag_consecutive_index(w, q);
  if (q < w.outside) {
    while (w.inside(col, io)) ++io;
    return w.src0 + io++;
  }
  while (!w.inside(col, ii)) ++ii;
  return w.src0 + ii++;
}

__device__ __forceinline__ bool same_bits(double x, double y) {
  return __double_as_longlong(x) == __double_as_longlong(y);
}

template <bool SHARED>
__global__ __launch_bounds__(kBlock) void wjag_plan_kernel(const int64_t *rp, const int32_t *col,
                                                           const double2 *val, int64_t n,
                                                           int32_t N, int64_t nwb, int32_t *wglob,
                                                           int32_t *wshn, int64_t *wcnt) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (k >= nwb) return;  // the whole wavefront leaves together
  const int64_t r0 = k * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, n - r0);
  const WjagRow w = wjag_row(rp, col, r0, nr, N, lane);
  // G = fewest outside entries of a non-empty row; the block is regular when
  // its rows share one rho-row and every row longer than G has exactly G
  int G = 1 << 30, gmin = 1 << 30;
  for (int j = 0; j < 64; ++j) {
    const int lj = __shfl(w.len, j, 64), oj = __shfl(w.outside, j, 64);
    if (lj > 0 && oj < G) G = oj;
    if (lj >= 0 && oj < gmin) gmin = oj;
  }
  if (G == (1 << 30)) G = 0;
  if (gmin == (1 << 30)) gmin = 0;
  const bool odd = w.len > G && w.outside != G;
  const bool regular = __ballot(odd) == 0 && r0 / N == (r0 + nr - 1) / N;
  // shared leading positions: same offset from the row and same real or
  // imaginary value in every row of the block
  int gs = 0;
  if constexpr (SHARED) {
    // is position q the same in every row? (entry of the lane's row given)
    auto same = [&](int64_t e_col, double2 v) {
      const int64_t rel = lane < nr ? e_col - w.row : 0;
      if (lane >= nr) v = make_double2(0.0, 0.0);
      const int64_t rel0 = __shfl(rel, 0, 64);
      const double vx0 = __shfl(v.x, 0, 64), vy0 = __shfl(v.y, 0, 64);
      const bool ok = lane >= nr || (rel == rel0 && same_bits(v.x, vx0) && same_bits(v.y, vy0) &&
                                     (v.x == 0.0 || v.y == 0.0));
      return __ballot(!ok) == 0;
    };
    if (__ballot(!w.consecutive) == 0) {
      // eight positions' loads in flight per step (gmin > 0: every row of
      // the block has entries)
      for (int q0 = 0; q0 < gmin && q0 < kSharedMax && gs == q0; q0 += 8) {
        int32_t cc[8];
        double2 vv[8];
        wjag_load8(col, val, w, q0, cc, vv);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (q0 + u >= gmin || gs != q0 + u) break;
          if (same((int64_t)cc[u], vv[u])) ++gs;
        }
      }
    } else {
      int io = 0, ii = 0;
      for (int q = 0; q < gmin && q < kSharedMax; ++q) {
        int64_t c = 0;
        double2 v = make_double2(0.0, 0.0);
        if (lane < nr) {
          const int64_t e = wjag_next(col, w, q, io, ii);
          c = (int64_t)col[e];
          v = val[e];
        }
        if (!same(c, v)) break;
        ++gs;
      }
    }
  }
  // In a regular block, is the entry at position G (the first inside entry,
  // at CSR index lo) every row's diagonal?  (Assembled rows put it first.)
  bool dfirst = false;
  if (regular) {
    const bool okd = lane >= nr || (w.len > G && (int64_t)col[w.src0 + w.lo] == w.row);
    dfirst = __ballot(!okd) == 0;
  }
  long long cnt = lane < nr ? (long long)(w.len - gs) : 0;
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) {
    wglob[k] = regular ? (G | (dfirst ? kGlobDiagFirst : 0)) : -1;
    wshn[k] = gs;
    wcnt[k] = cnt;
  }
}

template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void wjag_fill_kernel(
    const int64_t *rp, const int32_t *col, const double2 *val, int64_t n, int32_t N, int64_t nwb,
    const int32_t *wshn, const int64_t *wstart, const int64_t *wshs, int32_t *wcol, double2 *wval,
    double *wcoef, double2 *wdiag, int32_t *wlen, unsigned char *wperm, SharedEntry *wsh,
    int *bad) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (k >= nwb) return;
  const int64_t r0 = k * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, n - r0);
  const WjagRow w = wjag_row(rp, col, r0, nr, N, lane);
  int rank = 0;
  int maxlen = 0;
  for (int j = 0; j < 64; ++j) {
    const int lj = __shfl(w.len, j, 64);
    rank += (lj > w.len) || (lj == w.len && j < lane);
    maxlen = lj > maxlen ? lj : maxlen;
  }
  if (lane < nr) {
    wlen[r0 + rank] = w.len;
    wperm[r0 + rank] = (unsigned char)lane;
  }
  const int gs = wshn[k];
  const int64_t e0 = wstart[k];
  double2 dg = make_double2(0.0, 0.0);
  int ndiag = 0;
  bool mixed = false;
  int ps = 0;
  // the lane's entry at position p (w.len > p)
  auto put = [&](int p, int32_t cc, double2 vv) {
      if (p < gs) {  // the same in every row: lane 0 stores it for the block
        if (lane == 0) {
          const bool im = vv.x == 0.0 && vv.y != 0.0;
          wsh[wshs[k] + p] =
              SharedEntry{(int32_t)((int64_t)cc - w.row), im ? kImagBit : 0u, im ? vv.y : vv.x};
        }
      } else {
        const int64_t dst = e0 + ps + rank;
        const int32_t rel = (int32_t)((int64_t)cc - w.row);
        const uint32_t off = (uint32_t)rel & kOffMask;
        if constexpr (!SPLIT) {
          wcol[dst] = rel;
          wval[dst] = vv;
        } else if (cc == w.row) {
          dg = vv;
          ++ndiag;
          wcol[dst] = (int32_t)kDiagBit;
          wcoef[dst] = 0.0;
        } else if (vv.x != 0.0 && vv.y != 0.0) {
          mixed = true;
          wcol[dst] = (int32_t)off;
          wcoef[dst] = 0.0;
        } else if (vv.x == 0.0 && vv.y != 0.0) {
          wcol[dst] = (int32_t)(off | kImagBit);
          wcoef[dst] = vv.y;
        } else {
          wcol[dst] = (int32_t)off;
          wcoef[dst] = vv.x;
        }
      }
  };
  if (__ballot(!w.consecutive) == 0) {
    // eight positions' loads in flight per step (maxlen > 0: nnz > 0)
    for (int p0 = 0; p0 < maxlen; p0 += 8) {
      int32_t cc[8];
      double2 vv[8];
      wjag_load8(col, val, w, p0, cc, vv);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = p0 + u;
        if (p >= maxlen) break;
        const int cnt = __popcll(__ballot(w.len > p));
        if (w.len > p) put(p, cc[u], vv[u]);
        if (p >= gs) ps += cnt;
      }
    }
  } else {
    int io = 0, ii = 0;
    for (int p = 0; p < maxlen; ++p) {
      const int cnt = __popcll(__ballot(w.len > p));
      if (w.len > p) {
        const int64_t e = wjag_next(col, w, p, io, ii);
        put(p, col[e], val[e]);
      }
      if (p >= gs) ps += cnt;
    }
  }
  // zero entries up to the padded count
  if (lane == 0)
    for (int64_t q = wshs[k] + gs; q < wshs[k + 1]; ++q) wsh[q] = SharedEntry{0, 0u, 0.0};
  if constexpr (SPLIT) {
    if (lane < nr) wdiag[r0 + rank] = dg;
    if (mixed || ndiag > 1) *(volatile int *)bad = 1;
  }
}

// Blocks whose stored rows are word for word the same (after the shared
// positions, with columns as offsets from the row) can read one copy.  The
// hash covers each rank's remaining length and the block's stored words;
// equal hashes are then compared in full before a block is pointed at
// another's copy.
__device__ __forceinline__ unsigned long long mix64(unsigned long long h, unsigned long long v) {
  // SplitMix64 finaliser (Steele, Lea and Flood, 2014) of h ^ v
  unsigned long long z = h ^ v;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long value_word(const double *wcoef, const double2 *wval,
                                                         int64_t i, int half) {
  return (unsigned long long)__double_as_longlong(wcoef ? wcoef[i] : (half ? wval[i].y : wval[i].x));
}

__global__ __launch_bounds__(kBlock) void wjag_hash_kernel(const int32_t *wcol, const double *wcoef,
                                                           const double2 *wval, const int32_t *wlen,
                                                           const int32_t *wshn,
                                                           const int64_t *wstart, int64_t n,
                                                           int64_t nwb, unsigned long long *hash) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (k >= nwb) return;
  const int64_t r0 = k * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, n - r0);
  const int gs = wshn[k];
  unsigned long long h = mix64(0x51A7E5ull + lane, lane < nr ? (unsigned)(wlen[r0 + lane] - gs) : ~0u);
  for (int64_t i = wstart[k] + lane; i < wstart[k + 1]; i += 64) {
    h = mix64(h, (unsigned)wcol[i]);
    h = mix64(h, value_word(wcoef, wval, i, 0));
    if (!wcoef) h = mix64(h, value_word(wcoef, wval, i, 1));
  }
  for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
  if (lane == 0) hash[k] = h;
}

// same[k] = 1 when block k's stored rows equal those of block canon[k].
__global__ __launch_bounds__(kBlock) void wjag_same_kernel(const int32_t *wcol, const double *wcoef,
                                                           const double2 *wval, const int32_t *wlen,
                                                           const int32_t *wshn,
                                                           const int64_t *wstart, int64_t n,
                                                           int64_t nwb, const int64_t *canon,
                                                           int *same) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (k >= nwb) return;
  const int64_t c = canon[k];
  if (c == k) {
    if (lane == 0) same[k] = 0;
    return;
  }
  const int64_t r0 = k * kWaveRows, q0 = c * kWaveRows;
  const int nr = (int)min((int64_t)kWaveRows, n - r0), nq = (int)min((int64_t)kWaveRows, n - q0);
  bool diff = nr != nq || wstart[k + 1] - wstart[k] != wstart[c + 1] - wstart[c];
  if (!diff && lane < nr) diff = wlen[r0 + lane] - wshn[k] != wlen[q0 + lane] - wshn[c];
  const int64_t d = wstart[c] - wstart[k];
  if (__ballot(diff) == 0) {
    for (int64_t i = wstart[k] + lane; i < wstart[k + 1]; i += 64) {
      diff = diff || wcol[i] != wcol[i + d] ||
             value_word(wcoef, wval, i, 0) != value_word(wcoef, wval, i + d, 0) ||
             (!wcoef && value_word(wcoef, wval, i, 1) != value_word(wcoef, wval, i + d, 1));
    }
  }
  const bool any = __ballot(diff) != 0;
  if (lane == 0) same[k] = any ? 0 : 1;
}

// max over rows of sum_e |val[e]|  (on the adjoint this is ||L||_1).
// ||L||_1 as the largest row sum of |L^dagger| from the CSR of L (graph
// walks with a real H, whose rows are in structural order: the H rho
// entries, the diagonal, the rho H entries, then the population transfers):
// off the rows (a, a) a row of L^dagger holds the moduli of the row of L in
// the same order; a row (a, a) holds those of its first entries and then
// its own transfers (omega R_ja, ascending j; frp: the rates' row pointer of
// L, whose transfers it drops) - the sums, in the order of the assembled
// CSR of L^dagger, are bit for bit row_abs_max_kernel's on that CSR.
__global__ __launch_bounds__(kBlock) void adj_row_abs_max_kernel(
    int64_t n, int32_t N, const int64_t *rp, const double2 *val, const int64_t *frp,
    const int64_t *trp, const double *tval, unsigned long long *out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long m[1] = {0ull};
  if (r < n) {
    const int64_t a = r / N;
    const bool diag_row = r == a * ((int64_t)N + 1);
    double s = 0.0;
    const int64_t e0 = rp[r];
    const int64_t e1 = rp[r + 1] - (diag_row ? frp[a + 1] - frp[a] : 0);
    for (int64_t i0 = e0; i0 < e1; i0 += 8) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = val[min(i0 + u, e1 - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < e1) s += cabs2(v[u]);
    }
    if (diag_row)
      for (int64_t e = trp[a]; e < trp[a + 1]; ++e) s += cabs2(make_double2(tval[e], 0.0));
    m[0] = abs_bits(s);
  }
  unsigned long long *const dst[1] = {out};
  block_umax_to<1>(m, dst, nullptr);
}

__global__ __launch_bounds__(kBlock) void row_abs_max_kernel(int64_t n, const int64_t *rp,
                                                             const double2 *val,
                                                             unsigned long long *out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long m[1] = {0ull};
  if (r < n) {
    // entries in order; eight loads in flight per step
    double s = 0.0;
    const int64_t e0 = rp[r], e1 = rp[r + 1];
    for (int64_t i0 = e0; i0 < e1; i0 += 8) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = val[min(i0 + u, e1 - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < e1) s += cabs2(v[u]);
    }
    m[0] = abs_bits(s);
  }
  unsigned long long *const dst[1] = {out};
  block_umax_to<1>(m, dst, nullptr);
}

__global__ void zero_kernel(unsigned int *p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Round complex128 values to complex64 (to nearest, per component).
__global__ void to_c64_kernel(float2 *dst, const double2 *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

// Round doubles to float (to nearest).
__global__ void to_f32_kernel(float *dst, const double *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void copy_kernel(double2 *dst, const double2 *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// --------------------------------------------------------------------------
// Term j of one scaling step of the single-time algorithm.
// --------------------------------------------------------------------------

// Returns true when the step already passed the two-term test (then every
// workgroup of this launch returns at once).  Evaluated identically by every
// workgroup from values written by earlier launches.
__device__ __forceinline__ bool taylor_prologue(const SpmvArgs &a) {
  StepSlots *S = &a.st->step[a.par];
  bool stop = false;
  if (a.j >= 2) {
    // The flag and the norms were written by earlier launches, which the
    // kernel boundary makes visible: plain (cached) loads, issued together.
    // Coherent loads here would all queue at the memory side on the line
    // that this launch's norm atomics update.
    const int flag = S->stop;
    const double c1 = bits_to_d(a.j == 2 ? S->b0 : S->b[a.j - 2]);
    const double c2 = bits_to_d(S->b[a.j - 1]);
    const double f = bits_to_d(S->f[a.j - 1]);
    const bool pass = c1 + c2 <= a.tol * f;
    stop = (flag != 0) | pass;  // one branch on both loads
    // one writer: the rest of this launch reaches the same verdict itself,
    // and later launches see the flag across the kernel boundary
    if (!flag && pass && blockIdx.x == 0 && threadIdx.x == 0) S->stop = 1;
  } else if (blockIdx.x == 0) {
    // first term of a step: clear the other parity for the next step
    unsigned int *o = (unsigned int *)&a.st->step[a.par ^ 1];
    for (int i = threadIdx.x; i < (int)(sizeof(StepSlots) / 4); i += kBlock) o[i] = 0u;
  }
  // Paced launches: launch seq - 1 has ended when this one runs, and `stop`
  // says whether its step passed the test after it; posted to the host word
  // (which the host alone reads: no ordering of other writes is needed).
  if (a.progress && blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(a.progress, ((a.seq - 1) << 1) | (stop ? 1ull : 0ull), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  if (stop) return true;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.st->products, 1ull);
  return false;
}

template <int ENGINE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(term_waves(ENGINE)))) void term_kernel(SpmvArgs a) {
  if (taylor_prologue(a)) return;
  TaylorEpi epi(a);
  run_engine<ENGINE>(a, epi);
  StepSlots *S = &a.st->step[a.par];
  unsigned long long v[3] = {epi.mb, epi.mf, epi.mb0};
  unsigned long long *const dst[3] = {&S->b[a.j], &S->f[a.j], a.j == 1 ? &S->b0 : nullptr};
  block_umax_to<3>(v, dst, &a.st->nonfinite);
}

// ---------------------------------------------------------------------------
// Single-precision products (QSW_PREC_FP32).  The term is a complex64
// vector; the accumulator F is a pair of complex64 vectors whose unevaluated
// sum hi + lo carries about twice the float significand, so that adding m
// terms to it loses nothing beyond the terms' own rounding.  Norms, the
// stopping test and the parameters stay in double.
// ---------------------------------------------------------------------------

// s + e = a + b exactly (Knuth's two-sum; the build keeps every operation
// as written: no contraction, no reassociation).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) + y for one component: the two-sum of hi and y, its error folded
// into lo, then renormalised so that |lo| is at most half an ulp of hi.
__device__ __forceinline__ void df_add(float hi, float lo, float y, float &h2, float &l2) {
  float s, e;
  two_sum(hi, y, s, e);
  const float t = lo + e;
  h2 = s + t;
  l2 = t - (h2 - s);
}

__device__ __forceinline__ double cabs_df(float2 hi, float2 lo) {
  return cabs2(make_double2((double)hi.x + (double)lo.x, (double)hi.y + (double)lo.y));
}

struct Taylor32Epi {  // y = alpha A x (complex64) ; F_out = F_in + y (two-float) ; norms
  const SpmvArgs &a;
  unsigned long long mb = 0, mf = 0, mb0 = 0;
  struct Pre {
    float2 hi, lo;
  };
  __device__ explicit Taylor32Epi(const SpmvArgs &args) : a(args) {}
  __device__ __forceinline__ Pre pre(int64_t row) const {
    return Pre{gld(a.fin_hi + row), gld(a.fin_lo + row)};
  }
  __device__ __forceinline__ void operator()(int64_t row, const float *acc, Pre f) {
    // the row sum scaled in double and rounded once
    const float2 y = make_float2((float)(a.alpha * (double)acc[0]),
                                 (float)(a.alpha * (double)acc[1]));
    gst(a.y32 + row, y);
    if (a.j == 1) mb0 = umax(mb0, abs_bits(cabs_df(f.hi, f.lo)));
    float2 h, l;
    df_add(f.hi.x, f.lo.x, y.x, h.x, l.x);
    df_add(f.hi.y, f.lo.y, y.y, h.y, l.y);
    gst(a.fout_hi + row, h);
    gst(a.fout_lo + row, l);
    mb = umax(mb, abs_bits(cabs2(make_double2((double)y.x, (double)y.y))));
    mf = umax(mf, abs_bits(cabs_df(h, l)));
  }
};

// Engines of the single-precision products: the wave layouts' traversal 0
// (plain) or 1 (rho-row staged; the XCD-banded traversal runs staged), with
// complex (1) or phase-split (11) single-precision values.
template <int ENGINE, class Epi>
__device__ __forceinline__ void run_engine32(const SpmvArgs &a, Epi &epi) {
  constexpr int trav = ENGINE / 100, fmt = ENGINE % 100;
  static_assert(trav <= 1 && (fmt == 1 || fmt == 11), "single-precision engine");
  wave_engine<1, true, trav == 1, fmt == 11, Epi, true>(a, epi);
}

template <int ENGINE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(QSW_TERM32_WAVES))) void term32_kernel(SpmvArgs a) {
  if (taylor_prologue(a)) return;
  Taylor32Epi epi(a);
  run_engine32<ENGINE>(a, epi);
  StepSlots *S = &a.st->step[a.par];
  unsigned long long v[3] = {epi.mb, epi.mf, epi.mb0};
  unsigned long long *const dst[3] = {&S->b[a.j], &S->f[a.j], a.j == 1 ? &S->b0 : nullptr};
  block_umax_to<3>(v, dst, &a.st->nonfinite);
}

__global__ __launch_bounds__(kBlock) void split_c64_kernel(const double2 *v, float2 *hi,
                                                           float2 *lo, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double2 z = gld(v + i);
    const float2 h = make_float2((float)z.x, (float)z.y);
    gst(hi + i, h);
    gst(lo + i, make_float2((float)(z.x - (double)h.x), (float)(z.y - (double)h.y)));
  }
}

// One workgroup: the diagonal's sum in double, in a fixed order (strided
// partial sums, then a tree over the workgroup).
__global__ __launch_bounds__(kBlock) void trace32_kernel(DeviceState *st, const float2 *hi,
                                                         const float2 *lo, int32_t N,
                                                         int reference) {
  __shared__ double part[kBlock];
  double acc = 0.0;
  for (int64_t a = threadIdx.x; a < N; a += kBlock) {
    const int64_t i = a * (N + 1);
    acc += (double)gld(hi + i).x + (double)gld(lo + i).x;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tr = part[0];
    if (!isfinite(tr)) st->nonfinite = 1;
    if (reference) {
      st->tr0 = tr;
      st->scale = 1.0;
    } else {
      const double tr0 = st->tr0;
      // scaled only when the deviation is small: a traceless or nearly
      // traceless input keeps its values
      const bool ok = isfinite(tr) && isfinite(tr0) && tr != 0.0 && tr0 != 0.0 &&
                      fabs(tr - tr0) <= 0x1p-10 * fabs(tr0);
      st->scale = ok ? tr0 / tr : 1.0;
      const unsigned long long d = abs_bits(tr - tr0);
      if (d > st->trace_dev) st->trace_dev = d;
    }
  }
}

__global__ __launch_bounds__(kBlock) void emit32_kernel(const DeviceState *st, float2 *hi,
                                                        float2 *lo, double2 *out, int64_t n) {
  const double f = st->scale;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float2 h = gld(hi + i), l = gld(lo + i);
    const double2 z = make_double2(((double)h.x + (double)l.x) * f, ((double)h.y + (double)l.y) * f);
    gst(out + i, z);
    if (f != 1.0) {
      const float2 h2 = make_float2((float)z.x, (float)z.y);
      gst(hi + i, h2);
      gst(lo + i, make_float2((float)(z.x - (double)h2.x), (float)(z.y - (double)h2.y)));
    }
  }
}

template <int ENGINE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void plain_kernel(SpmvArgs a) {
  PlainEpi epi(a);
  run_engine<ENGINE>(a, epi);
}

// --------------------------------------------------------------------------
// Time-series branch: powers K_p = (h/p) A K_{p-1} formed lazily, and the
// point sums F_k = Z + sum_p k^p K_p with the two-term stopping test.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void vec_norm_kernel(const double2 *x, int64_t n,
                                                          unsigned long long *dst) {
  unsigned long long m[1] = {0ull};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    m[0] = umax(m[0], abs_bits(cabs2(x[i])));
  unsigned long long *const d[1] = {dst};
  block_umax_to<1>(m, d, nullptr);
}

// Has point k already passed the test after term p-1?  (Evaluated the same
// way by every workgroup from values written by earlier launches.)
__device__ __forceinline__ bool point_done(const DeviceState *st, PointSlots *pt, int k, int p,
                                           double tol) {
  // flags and norms come from earlier launches: plain loads (see taylor_prologue)
  if (pt->stop) return true;
  if (p < 2) return false;
  const int q = p - 1;  // last term added
  const double kk = (double)k;
  const double c1 = (q == 1) ? bits_to_d(st->series.kn[0])
                             : pow(kk, (double)(q - 1)) * bits_to_d(st->series.kn[q - 1]);
  const double c2 = pow(kk, (double)q) * bits_to_d(st->series.kn[q]);
  if (c1 + c2 <= tol * bits_to_d(pt->f[q])) {
    if (blockIdx.x == 0 && threadIdx.x == 0) pt->stop = 1;  // one writer
    return true;
  }
  return false;
}

template <int ENGINE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void series_power_kernel(SpmvArgs a, PointSlots *pt, int k,
                                                              int p) {
  if (point_done(a.st, pt, k, p, a.tol)) return;
  if (p <= a.st->series.mhat) return;  // K_p already formed (by an earlier launch)
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.st->products, 1ull);
  PowerEpi epi(a);
  run_engine<ENGINE>(a, epi);
  unsigned long long v[1] = {epi.mk};
  unsigned long long *const dst[1] = {&a.st->series.kn[p]};
  block_umax_to<1>(v, dst, &a.st->nonfinite);
}

__global__ __launch_bounds__(kBlock) void series_accum_kernel(DeviceState *st, PointSlots *pt,
                                                              int k, int p, const double2 *Kp,
                                                              const double2 *Z, double2 *F,
                                                              int64_t n, double tol) {
  if (pt->stop) return;  // set by an earlier launch
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&st->series.mhat, p);
  const double kp = pow((double)k, (double)p);
  unsigned long long mf[1] = {0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double2 kv = Kp[i];
    double2 f = (p == 1) ? Z[i] : F[i];
    f.x = fma(kp, kv.x, f.x);
    f.y = fma(kp, kv.y, f.y);
    F[i] = f;
    mf[0] = umax(mf[0], abs_bits(cabs2(f)));
  }
  unsigned long long *const dst[1] = {&pt->f[p]};
  block_umax_to<1>(mf, dst, &st->nonfinite);
}

// --------------------------------------------------------------------------
// ADJ products: the rows (a, a) of L^dagger, one wavefront each, from the
// CSR of L (structural row order: H rho entries, diagonal, rho H entries,
// then the transfers of L, which are dropped) and the transposed rates.  The
// terms go in the order and form of the assembled L^dagger's phase-split
// layout, where the row's H rho entries and its own transfers are its
// entries outside its rho-row and come first, then the diagonal and the
// rho H entries: each a complex multiply-add with the value (0, coef),
// (coef, 0) or the diagonal.  The lanes fetch 64 terms at a time; every
// lane then takes them in order from the lanes (readlane), so the sums are
// that layout's (up to the sign of a zero) and reach the same epilogue.
__device__ __forceinline__ double rdl(double v, int l) {
  const long long u = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int NRHS, class Epi>
__device__ __forceinline__ void adj_diag_row(const SpmvArgs &a, int64_t ra, Epi &epi) {
  const int lane = threadIdx.x & 63;
  const int64_t N = a.N, row = ra * (N + 1);
  const int64_t e0 = a.rp[row], e1 = a.rp[row + 1];
  const int64_t t0 = a.trp[ra], t1 = a.trp[ra + 1];
  // the diagonal (ed; always stored) and the end of the rho H entries (er)
  int64_t ed = e1, er = e1;
  for (int64_t b = e0; b < e1 && ed == e1; b += 64) {
    const int64_t e = b + lane;
    const unsigned long long m = __ballot(e < e1 && (int64_t)a.col[e] == row);
    if (m) ed = b + __ffsll((long long)m) - 1;
  }
  for (int64_t b = ed + 1; b < e1 && er == e1; b += 64) {
    const int64_t e = b + lane;
    const unsigned long long m = __ballot(e < e1 && (int64_t)a.col[e] / N != ra);
    if (m) er = b + __ffsll((long long)m) - 1;
  }
  const int64_t nh = ed - e0, nt = t1 - t0;
  const int64_t terms = ed < e1 ? nh + nt + 1 + (er - ed - 1) : nh + nt;
  double acc[2 * NRHS];
#pragma unroll
  for (int q = 0; q < 2 * NRHS; ++q) acc[q] = 0.0;
  for (int64_t b = 0; b < terms; b += 64) {
    // term q = b + lane: value and column
    const int64_t q = b + lane;
    double2 v = make_double2(0.0, 0.0);
    int64_t c = row;
    if (q < terms) {
      if (q < nh) {
        v = make_double2(0.0, -a.val[e0 + q].y);
        c = a.col[e0 + q];
      } else if (q < nh + nt) {
        v = make_double2(a.tval[t0 + q - nh], 0.0);
        c = (int64_t)a.tcol[t0 + q - nh] * (N + 1);
      } else if (q == nh + nt) {
        const double2 d = a.val[ed];
        v = make_double2(d.x, -d.y);
      } else {
        const int64_t e = ed + 1 + (q - nh - nt - 1);
        v = make_double2(0.0, -a.val[e].y);
        c = a.col[e];
      }
    }
    double2 xq[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) xq[r] = a.x[c * NRHS + r];
    const int cnt = (int)min((int64_t)64, terms - b);
    for (int i = 0; i < cnt; ++i) {
      const double2 vi = make_double2(rdl(v.x, i), rdl(v.y, i));
#pragma unroll
      for (int r = 0; r < NRHS; ++r)
        cmac(acc[2 * r], acc[2 * r + 1], vi, make_double2(rdl(xq[r].x, i), rdl(xq[r].y, i)));
    }
  }
  if (lane == 0) epi(row, acc, typename Epi::Pre{});
}

// The ADJ product kernels' last workgroups (from a.adj_grid on) take the rows
// (a, a), one per wavefront; true for them.
template <int NRHS, class Epi>
__device__ __forceinline__ bool adj_diag_rows(const SpmvArgs &a, Epi &epi) {
  if ((int)blockIdx.x < a.adj_grid) return false;
  const int64_t ra = (int64_t)(blockIdx.x - a.adj_grid) * (kBlock / 64) + (threadIdx.x >> 6);
  if (ra < a.N) adj_diag_row<NRHS>(a, ra, epi);
  return true;
}

// Two right-hand sides (block 1-norm estimation) through the wave layout;
// ADJ: products with L^dagger through the layout of L.
// --------------------------------------------------------------------------
template <bool SPLIT, bool STAGE, bool ADJ = false>
__global__ __launch_bounds__(kBlock) void spmm2_kernel(SpmvArgs a, int mode, double *part,
                                                       double2 *sgn, double *h) {
  Spmm2Epi epi{a.y, mode, sgn, h};
  if constexpr (ADJ)
    if (adj_diag_rows<2>(a, epi)) return;
  wave_engine<2, false, STAGE, SPLIT, Spmm2Epi, false, ADJ>(a, epi, ADJ ? a.adj_grid : 0);
  if (mode == 1) {
    // deterministic per-workgroup column sums: fixed tree over the threads
    __shared__ double sm0[kBlock], sm1[kBlock];
    sm0[threadIdx.x] = epi.s0;
    sm1[threadIdx.x] = epi.s1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        sm0[threadIdx.x] += sm0[threadIdx.x + w];
        sm1[threadIdx.x] += sm1[threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = sm0[0];
      part[2 * blockIdx.x + 1] = sm1[0];
    }
  }
}

// Merged power chains of the 1-norm estimator (see WideOut): nr interleaved
// columns, no staging (the rho-rows of many columns do not fit the LDS).
// The per-column sums are the two-column product's, in the same order, and
// the finishing pair's epilogue and per-workgroup column sums are the same
// as spmm2_kernel's with the same grid.
template <int NR>
struct WideEpi {
  WideOut o;
  double s0 = 0.0, s1 = 0.0;
  typedef NoPre Pre;
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre) {
#pragma unroll
    for (int c = 0; c < NR; ++c)
      if (c < o.ys) o.Y[row * o.ys + c] = make_double2(acc[2 * c], acc[2 * c + 1]);
    if (o.fin) {
      const double2 y0 = make_double2(acc[2 * NR - 4], acc[2 * NR - 3]);
      const double2 y1 = make_double2(acc[2 * NR - 2], acc[2 * NR - 1]);
      const double m0 = cabs2(y0), m1 = cabs2(y1);
      if (o.mode == 1) {
        s0 += m0;
        s1 += m1;
        o.sgn[2 * row] = m0 > 0.0 ? make_double2(y0.x / m0, y0.y / m0) : make_double2(1.0, 0.0);
        o.sgn[2 * row + 1] =
            m1 > 0.0 ? make_double2(y1.x / m1, y1.y / m1) : make_double2(1.0, 0.0);
      } else if (o.mode == 2) {
        o.h[row] = m0 > m1 ? m0 : m1;
      }
    }
  }
};

template <bool SPLIT, int NR, bool ADJ = false>
__global__ __launch_bounds__(kBlock) void spmm_wide_kernel(SpmvArgs a, WideOut o) {
  WideEpi<NR> epi{o};
  if constexpr (ADJ)
    if (adj_diag_rows<NR>(a, epi)) return;
  wave_engine<NR, false, false, SPLIT, WideEpi<NR>, false, ADJ>(a, epi, ADJ ? a.adj_grid : 0);
  if (o.fin && o.mode == 1) {
    __shared__ double sm0[kBlock], sm1[kBlock];
    sm0[threadIdx.x] = epi.s0;
    sm1[threadIdx.x] = epi.s1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        sm0[threadIdx.x] += sm0[threadIdx.x + w];
        sm1[threadIdx.x] += sm1[threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      o.part[2 * blockIdx.x] = sm0[0];
      o.part[2 * blockIdx.x + 1] = sm1[0];
    }
  }
}


__global__ void pack_pairs_kernel(double2 *W, int64_t n, PairSources ps) {
  const int c = 2 * ps.chains;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int j = 0; j < ps.chains; ++j) {
      const double2 a = ps.src[j][2 * i], b = ps.src[j][2 * i + 1];
      W[i * c + 2 * j] = a;
      W[i * c + 2 * j + 1] = b;
    }
  }
}

__global__ void unit_pairs_kernel(double2 *W, int64_t n, PairUnits pu) {
  const int c = 2 * pu.chains;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int j = 0; j < pu.chains; ++j) {
      W[i * c + 2 * j] = make_double2(i == pu.ind[j][0] ? 1.0 : 0.0, 0.0);
      W[i * c + 2 * j + 1] = make_double2(i == pu.ind[j][1] ? 1.0 : 0.0, 0.0);
    }
  }
}

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double *part, int nb,
                                                              double *out2) {
  __shared__ double sm0[kBlock], sm1[kBlock];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  sm0[threadIdx.x] = s0;
  sm1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sm0[threadIdx.x] += sm0[threadIdx.x + w];
      sm1[threadIdx.x] += sm1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = sm0[0];
    out2[1] = sm1[0];
  }
}

// Probe block of the 1-norm estimator: column 0 = 1/n, column 1 = s_i / n
// with s_0 = -1 and s_i (i > 0) the sign of the top bit of SplitMix64
// (Steele, Lea and Flood, 2014) of 0x51A7E5 + i; column 1 is zero when t = 1.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void probe_init_kernel(double2 *X, int64_t n, int t) {
  const double inv = 1.0 / (double)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    X[2 * i] = make_double2(inv, 0.0);
    double sg = (splitmix64(0x51A7E5ull + (unsigned long long)i) >> 63) ? -1.0 : 1.0;
    if (i == 0) sg = -1.0;
    X[2 * i + 1] = make_double2(t == 2 ? sg * inv : 0.0, 0.0);
  }
}

// X = [e_i0, e_i1] (i1 < 0: second column zero).
__global__ void unit_cols_kernel(double2 *X, int64_t n, int64_t i0, int64_t i1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    X[2 * i] = make_double2(i == i0 ? 1.0 : 0.0, 0.0);
    X[2 * i + 1] = make_double2(i == i1 ? 1.0 : 0.0, 0.0);
  }
}

// dst = src with the two interleaved columns of every row exchanged.
__global__ void swap_pairs_kernel(double2 *dst, const double2 *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 u = src[2 * i], v = src[2 * i + 1];
    dst[2 * i] = v;
    dst[2 * i + 1] = u;
  }
}

// Total order of the estimator's candidates: larger h first, then smaller index.
__device__ __forceinline__ bool cand_better(double va, int64_t ia, double vb, int64_t ib) {
  return va > vb || (va == vb && ia < ib);
}

// Block argmax of (value, index) pairs by cand_better; every thread gets the
// winner.  red_v / red_i hold kBlock entries.
__device__ __forceinline__ void block_best(double &v, int64_t &i, double *red_v, int64_t *red_i) {
  red_v[threadIdx.x] = v;
  red_i[threadIdx.x] = i;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ov = red_v[threadIdx.x + w];
      const int64_t oi = red_i[threadIdx.x + w];
      if (cand_better(ov, oi, red_v[threadIdx.x], red_i[threadIdx.x])) {
        red_v[threadIdx.x] = ov;
        red_i[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  v = red_v[0];
  i = red_i[0];
  __syncthreads();
}

// Top K of h[0..n) under cand_better, per workgroup over a strided share:
// K rounds, each excluding the winners of earlier rounds.
__global__ __launch_bounds__(kBlock) void topk_partial_kernel(const double *h, int64_t n, int K,
                                                              double *cand_v, int64_t *cand_i) {
  __shared__ double red_v[kBlock];
  __shared__ int64_t red_i[kBlock];
  __shared__ int64_t chosen[kTopKMax];
  for (int r = 0; r < K; ++r) {
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= chosen[q] == i;
      if (!taken && cand_better(h[i], i, bv, bi)) {
        bv = h[i];
        bi = i;
      }
    }
    block_best(bv, bi, red_v, red_i);
    if (threadIdx.x == 0) {
      chosen[r] = bi;
      cand_v[(int64_t)blockIdx.x * K + r] = bv;
      cand_i[(int64_t)blockIdx.x * K + r] = bi;
    }
    __syncthreads();
  }
}

// Merge the per-workgroup candidates into the global top K (one workgroup).
__global__ __launch_bounds__(kBlock) void topk_merge_kernel(const double *cand_v,
                                                            const int64_t *cand_i, int64_t m, int K,
                                                            double *out_v, int64_t *out_i) {
  __shared__ double red_v[kBlock];
  __shared__ int64_t red_i[kBlock];
  __shared__ int64_t chosen[kTopKMax];
  for (int r = 0; r < K; ++r) {
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t j = threadIdx.x; j < m; j += kBlock) {
      const int64_t i = cand_i[j];
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= chosen[q] == i;
      if (!taken && cand_better(cand_v[j], i, bv, bi)) {
        bv = cand_v[j];
        bi = i;
      }
    }
    block_best(bv, bi, red_v, red_i);
    if (threadIdx.x == 0) {
      chosen[r] = bi;
      out_v[r] = bv;
      out_i[r] = bi;
    }
    __syncthreads();
  }
}

__global__ void populations_kernel(const double2 *rho, int32_t N, int32_t count, double *pops) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * count;
  if (i >= total) return;
  const int64_t k = i / N, a = i - k * N;
  pops[i] = rho[k * (int64_t)N * N + a * N + a].x;
}

inline int blocks_for(int64_t n, int per = kBlock) {
  int64_t b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

// --------------------------------------------------------------------------
// Batched propagation.  Each cycle is one launch of batch_control_kernel
// (one thread per walk: take in the maxima of the op that just ran, apply
// the stopping tests, choose the walk's next op) and one launch of
// batch_work_kernel (every wave block of every active walk carries out its
// walk's op).  Each column of a walk goes through exactly the operations of
// qsw_propagate on that column alone: same terms, same sums in the same
// order, same tests.
// --------------------------------------------------------------------------
enum BatchPc : int32_t {
  PC_LOAD = 0,
  PC_START,
  PC_TERMS,
  PC_EMIT,
  PC_AFTER_EMIT,
  PC_SBLOCK,
  PC_SPOINT0,
  PC_SPOINT,
  PC_SAFTER_EMIT,
  PC_TREF,   // single-precision products: reference trace after the load
  PC_EMIT2   //   the emission after the point's trace check
};

__device__ void batch_issue_term(const BatchInst &I, const BatchCtl &C, BatchOp &O) {
  const int i = C.i, j = C.j, s = C.sseg;
  const double2 *src = (i == 0) ? I.V[C.cur] : I.F[(i - 1) & 1];
  double2 *dst = (i == s - 1) ? I.V[C.cur ^ 1] : I.F[i & 1];
  O.type = BOP_TERM;
  O.active = C.active;
  O.first = (j == 1);
  O.alpha = C.tseg / ((double)s * (double)j);
  O.x = (j == 1) ? src : I.B[(j - 1) & 1];
  O.y = I.B[j & 1];
  O.fin = (j == 1) ? src : dst;
  O.fout = dst;
}

// Single-precision products: term j of the scaling step from state pair
// `cur` into the other pair (as qsw_propagate's single-precision steps).
__device__ void batch_issue_term32(const BatchInst &I, const BatchCtl &C, BatchOp &O) {
  const int j = C.j, src = C.cur, dst = C.cur ^ 1;
  O.type = BOP_TERM;
  O.active = C.active;
  O.first = (j == 1);
  O.alpha = C.tseg / ((double)C.sseg * (double)j);
  O.x32 = (j == 1) ? I.Ph[src] : I.B32[(j - 1) & 1];
  O.y32 = I.B32[j & 1];
  O.fin_hi = (j == 1) ? I.Ph[src] : I.Ph[dst];
  O.fin_lo = (j == 1) ? I.Pl[src] : I.Pl[dst];
  O.fout_hi = I.Ph[dst];
  O.fout_lo = I.Pl[dst];
}

__device__ void batch_issue(const BatchInst &I, const BatchCtl &C, BatchOp &O) {
  if (I.prec32)
    batch_issue_term32(I, C, O);
  else
    batch_issue_term(I, C, O);
}

__device__ void batch_issue_series(const BatchInst &I, const BatchCtl &C, BatchOp &O) {
  const double2 *Z = I.V[C.cur];
  double2 *Fk = I.V[C.cur ^ 1];
  double2 *Kp = I.K + (int64_t)(C.p - 1) * I.vlen;
  O.active = C.active;
  O.first = (C.p == 1);
  O.kpow = pow((double)C.kk, (double)C.p);
  O.fin = (C.p == 1) ? Z : Fk;
  O.fout = Fk;
  if (C.p > C.mhat) {
    O.type = BOP_POWACC;
    O.x = (C.p == 1) ? Z : I.K + (int64_t)(C.p - 2) * I.vlen;
    O.y = Kp;
    O.alpha = I.dt / (double)C.p;
  } else {
    O.type = BOP_ACC;
    O.x = Kp;
    O.y = nullptr;
  }
}

__device__ void batch_start_segment(BatchCtl &C, int seg, double t, int m, int s, uint32_t all) {
  C.seg = seg;
  C.tseg = t;
  C.mseg = m;
  C.sseg = s;
  C.i = 0;
  C.j = 1;
  C.active = all;
}

__device__ void batch_advance(const BatchInst &I, BatchCtl &C, BatchOp &O, BatchSlots &S) {
  const uint32_t all = (1u << I.n0) - 1u;
  double y[kBatchMaxRhs], f[kBatchMaxRhs], b0[kBatchMaxRhs];
  bool bad = false;
  for (int c = 0; c < kBatchMaxRhs; ++c) {
    if (c < I.n0) bad |= (S.y[c] >= kInfBits) || (S.f[c] >= kInfBits) || (S.b0[c] >= kInfBits);
    y[c] = bits_to_d(S.y[c]);
    f[c] = bits_to_d(S.f[c]);
    b0[c] = bits_to_d(S.b0[c]);
    S.y[c] = 0ull;
    S.f[c] = 0ull;
    S.b0[c] = 0ull;
  }
  if (bad) C.nonfinite = 1;
  switch (C.last) {
    case BOP_TERM:
      for (int c = 0; c < kBatchMaxRhs; ++c) {
        if (!((C.active >> c) & 1u)) continue;
        C.c_prev[c] = (C.j == 1) ? b0[c] : C.c_last[c];
        C.c_last[c] = y[c];
        C.f_last[c] = f[c];
      }
      ++C.products;
      break;
    case BOP_POWACC:
      for (int c = 0; c < kBatchMaxRhs; ++c) I.kn[C.p * kBatchMaxRhs + c] = y[c];
      C.mhat = C.p;
      ++C.products;
      [[fallthrough]];
    case BOP_ACC:
      for (int c = 0; c < kBatchMaxRhs; ++c)
        if ((C.active >> c) & 1u) C.f_last[c] = f[c];
      break;
    case BOP_NORM:
      for (int c = 0; c < kBatchMaxRhs; ++c) I.kn[c] = b0[c];
      break;
    case BOP_TRACE:
      C.trace_dev = C.trace_dev > S.trace_dev ? C.trace_dev : S.trace_dev;
      break;
    default:
      break;
  }
  O.type = BOP_NONE;
  C.last = BOP_NONE;
  for (;;) {
    switch (C.pc) {
      case PC_LOAD:
        O.type = BOP_LOAD;
        C.pc = I.prec32 ? PC_TREF : PC_START;
        C.last = BOP_LOAD;
        return;
      case PC_TREF:  // the loaded state's trace: every later point's reference
        O.type = BOP_TRACE;
        O.first = 1;
        O.fout_hi = I.Ph[0];
        O.fout_lo = I.Pl[0];
        C.pc = PC_START;
        C.last = BOP_TRACE;
        return;
      case PC_START:
        if (I.t0 != 0.0 && I.m0 > 0) {
          batch_start_segment(C, 0, I.t0, I.m0, I.s0, all);
          batch_issue(I, C, O);
          C.pc = PC_TERMS;
          C.last = BOP_TERM;
          return;
        }
        C.point = 0;
        C.pc = PC_EMIT;
        continue;
      case PC_TERMS: {
        if (C.j < C.mseg) {
          uint32_t act = 0;
          for (int c = 0; c < kBatchMaxRhs; ++c)
            if (((C.active >> c) & 1u) && !(C.c_prev[c] + C.c_last[c] <= I.tol * C.f_last[c]))
              act |= 1u << c;
          if (act) {
            C.active = act;
            ++C.j;
            batch_issue(I, C, O);
            C.last = BOP_TERM;
            return;
          }
        }
        // the scaling step is complete (single-precision products: its
        // accumulator pair is the state from now on)
        if (I.prec32) C.cur ^= 1;
        ++C.i;
        if (C.i < C.sseg) {
          C.j = 1;
          C.active = all;
          batch_issue(I, C, O);
          C.last = BOP_TERM;
          return;
        }
        if (!I.prec32) C.cur ^= 1;  // the segment is complete
        C.point = (C.seg == 0) ? 0 : C.point + 1;
        C.pc = PC_EMIT;
        continue;
      }
      case PC_EMIT:
        // single-precision products: the trace check first, except for
        // point 0 at t0 = 0 (rho0 itself is emitted)
        if (I.prec32 && !(C.point == 0 && I.t0 == 0.0)) {
          O.type = BOP_TRACE;
          O.first = 0;
          O.fout_hi = I.Ph[C.cur];
          O.fout_lo = I.Pl[C.cur];
          C.pc = PC_EMIT2;
          C.last = BOP_TRACE;
          return;
        }
        [[fallthrough]];
      case PC_EMIT2:
        O.type = BOP_EMIT;
        O.point = C.point;
        O.x = I.V[C.cur];
        if (I.prec32) {
          O.first = (C.point == 0 && I.t0 == 0.0) ? 1 : 0;  // 1: copy rho0
          O.fout_hi = I.Ph[C.cur];
          O.fout_lo = I.Pl[C.cur];
        }
        C.pc = PC_AFTER_EMIT;
        C.last = BOP_EMIT;
        return;
      case PC_AFTER_EMIT:
        if (C.point >= I.q) {
          C.done = 1;
          return;
        }
        if (I.branch == 0) {
          if (I.m == 0) {  // exp(dt L) acts as the identity
            ++C.point;
            C.pc = PC_EMIT;
            continue;
          }
          batch_start_segment(C, 1, I.dt, I.m, I.s, all);
          batch_issue(I, C, O);
          C.pc = PC_TERMS;
          C.last = BOP_TERM;
          return;
        }
        C.blk = 1;
        C.zi = 0;
        C.pc = PC_SBLOCK;
        continue;
      case PC_SBLOCK:
        C.dd = (C.blk <= I.jb) ? I.d : I.r;
        if (C.dd == 0 || C.zi >= I.q) {
          C.done = 1;
          return;
        }
        O.type = BOP_NORM;
        O.x = I.V[C.cur];
        C.mhat = 0;
        C.pc = PC_SPOINT0;
        C.last = BOP_NORM;
        return;
      case PC_SPOINT0:
        C.kk = 1;
        C.p = 1;
        C.active = all;
        batch_issue_series(I, C, O);
        C.last = O.type;
        C.pc = PC_SPOINT;
        return;
      case PC_SPOINT: {
        if (C.p < I.m) {
          const int qq = C.p;
          const double kk = (double)C.kk;
          uint32_t act = 0;
          for (int c = 0; c < kBatchMaxRhs; ++c) {
            if (!((C.active >> c) & 1u)) continue;
            const double c1 = (qq == 1) ? I.kn[c]
                                        : pow(kk, (double)(qq - 1)) * I.kn[(qq - 1) * kBatchMaxRhs + c];
            const double c2 = pow(kk, (double)qq) * I.kn[qq * kBatchMaxRhs + c];
            if (!(c1 + c2 <= I.tol * C.f_last[c])) act |= 1u << c;
          }
          if (act) {
            C.active = act;
            ++C.p;
            batch_issue_series(I, C, O);
            C.last = O.type;
            return;
          }
        }
        O.type = BOP_EMIT;  // the point is complete
        O.point = C.zi + C.kk;
        O.x = I.V[C.cur ^ 1];
        C.pc = PC_SAFTER_EMIT;
        C.last = BOP_EMIT;
        return;
      }
      case PC_SAFTER_EMIT:
        if (C.kk < C.dd) {
          ++C.kk;
          C.p = 1;
          C.active = all;
          batch_issue_series(I, C, O);
          C.last = O.type;
          C.pc = PC_SPOINT;
          return;
        }
        C.cur ^= 1;  // the block's last point starts the next block
        C.zi += C.dd;
        ++C.blk;
        C.pc = PC_SBLOCK;
        continue;
      default:
        C.done = 1;
        return;
    }
  }
}

// One workgroup: walks b = tid, tid + kBlock, ...; writes the number still
// running to *live.
__global__ __launch_bounds__(kBlock) void batch_control_kernel(BatchArgs A) {
  __shared__ unsigned int cnt[kWaves];
  unsigned int alive = 0;
  for (int b = threadIdx.x; b < A.count; b += kBlock) {
    BatchCtl C = A.ctl[b];
    if (!C.done) {
      BatchOp O = A.op[b];
      batch_advance(A.inst[b], C, O, A.slots[b]);
      A.op[b] = O;
      A.ctl[b] = C;
      if (C.nonfinite) *(volatile int *)A.nonfinite = 1;
    } else {
      A.op[b].type = BOP_NONE;
    }
    alive += C.done ? 0u : 1u;
  }
  for (int off = 32; off > 0; off >>= 1) alive += __shfl_xor(alive, off, 64);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = alive;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int t = 0;
    for (int w = 0; w < kWaves; ++w) t += cnt[w];
    *A.live = t;
  }
}

template <int R>
struct BatchTermEpi {  // TERM and POWACC: y = alpha A x; accumulate active columns
  int64_t n;             // column stride of the vectors
  double alpha, kpow;
  const double2 *fin;
  double2 *fout, *y;
  uint32_t active;
  bool first, series;
  unsigned long long my[R], mf[R], mb0[R];
  typedef NoPre Pre;
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const double *acc, Pre) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 yv = make_double2(alpha * acc[2 * r], alpha * acc[2 * r + 1]);
      gst(y + r * n + row, yv);
      my[r] = umax(my[r], abs_bits(cabs2(yv)));
      if ((active >> r) & 1u) {
        double2 f = gld(fin + r * n + row);
        if (series) {
          f.x = fma(kpow, yv.x, f.x);
          f.y = fma(kpow, yv.y, f.y);
        } else {
          if (first) mb0[r] = umax(mb0[r], abs_bits(cabs2(f)));
          f.x += yv.x;
          f.y += yv.y;
        }
        gst(fout + r * n + row, f);
        mf[r] = umax(mf[r], abs_bits(cabs2(f)));
      }
    }
  }
};


// Single-precision products: y = alpha A x in complex64 (the row sum scaled
// in double and rounded once), added by two-sum to the active columns' hi +
// lo accumulator pairs; the norms as in Taylor32Epi.
template <int R>
struct BatchTerm32Epi {
  int64_t n;  // column stride of the vectors
  double alpha;
  const float2 *fin_hi, *fin_lo;
  float2 *fout_hi, *fout_lo, *y;
  uint32_t active;
  bool first;
  unsigned long long my[R], mf[R], mb0[R];
  typedef NoPre Pre;
  __device__ __forceinline__ Pre pre(int64_t) const { return Pre{}; }
  __device__ __forceinline__ void operator()(int64_t row, const float *acc, Pre) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float2 yv = make_float2((float)(alpha * (double)acc[2 * r]),
                                    (float)(alpha * (double)acc[2 * r + 1]));
      gst(y + r * n + row, yv);
      my[r] = umax(my[r], abs_bits(cabs2(make_double2((double)yv.x, (double)yv.y))));
      if ((active >> r) & 1u) {
        const float2 fh = gld(fin_hi + r * n + row), fl = gld(fin_lo + r * n + row);
        if (first) mb0[r] = umax(mb0[r], abs_bits(cabs_df(fh, fl)));
        float2 h, l;
        df_add(fh.x, fl.x, yv.x, h.x, l.x);
        df_add(fh.y, fl.y, yv.y, h.y, l.y);
        gst(fout_hi + r * n + row, h);
        gst(fout_lo + r * n + row, l);
        mf[r] = umax(mf[r], abs_bits(cabs_df(h, l)));
      }
    }
  }
};

// Tr of a state pair by one wavefront, in trace32_kernel's order: kBlock
// strided partial sums (lane l holds those of threads l + 64 q), then the
// same tree (levels of 64 and more within the lanes, the rest across them).
// Every lane returns the sum.
__device__ double wave_trace(const float2 *hi, const float2 *lo, int32_t N) {
  constexpr int Q = kBlock / 64 > 0 ? kBlock / 64 : 1;
  const int l = threadIdx.x & 63;
  double p[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double acc = 0.0;
    for (int64_t a = l + 64 * q; a < N; a += kBlock) {
      const int64_t i = a * (N + 1);
      acc += (double)gld(hi + i).x + (double)gld(lo + i).x;
    }
    p[q] = acc;
  }
#pragma unroll
  for (int w = kBlock / 2; w >= 64; w >>= 1) {
    const int wq = w / 64;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (q < wq) p[q] += p[q + wq];
  }
  double v = p[0];
  for (int w = 32; w >= 1; w >>= 1) {
    const double o = __shfl_down(v, w, 64);
    if (l < w) v += o;
  }
  return __shfl(v, 0, 64);
}

// xs[r N0 + c] = x0[r n0r + base + c] (all R columns), four loads per thread
// in flight before their LDS writes (one round trip per 4 kBlock elements
// instead of per kBlock; more would cost registers here).
template <int R, class T>
__device__ __forceinline__ void batch_stage(T *xs, const T *x0, int64_t n0r, int64_t base,
                                            int N0) {
  const int cnt = R * N0;
  for (int i0 = threadIdx.x; i0 < cnt; i0 += 4 * kBlock) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min(i0 + u * kBlock, cnt - 1);
      const int r = i / N0;
      v[u] = gld(x0 + (int64_t)r * n0r + base + (i - r * N0));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * kBlock < cnt) xs[i0 + u * kBlock] = v[u];
  }
}

__device__ __forceinline__ void batch_flush(unsigned long long v, unsigned long long *dst) {
  v = wave_umax(v);
  if ((threadIdx.x & 63) == 0 && v) atomicMax(dst, v);
}

// Global block g -> (walk, block within the walk), rebuilt when the set of
// running walks changes.
__global__ void batch_blocks_kernel(BatchArgs A) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.nblocks;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = A.nact;  // blk_start[lo] <= g < blk_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (A.blk_start[mid] <= g) lo = mid; else hi = mid;
    }
    A.blkmap[g] = make_int2(A.act[lo], (int)(g - A.blk_start[lo]));
  }
}

// Staging of the rho-row for the rho-H gathers (as in the single-walk
// engine, for all R columns): decided per workgroup from the walk of its
// first block, used by the waves whose block belongs to that walk.
// P32: the walks with single-precision products (the others skip theirs);
// a cycle with walks of both kinds launches both kernels.
template <int R, bool P32>
__global__ __launch_bounds__(kBlock, (R >= 2 ? 4 : 1)) void batch_work_kernel(BatchArgs A) {
  constexpr int WPB = kBlock / 64;
  extern __shared__ double2 xs[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t total = A.nblocks;
  // Each workgroup takes one contiguous run of block quads, so consecutive
  // iterations mostly stay within one walk and its data stays in the caches.
  // (Claiming quads from one shared counter was slower: its atomics
  // serialise.)
  const int64_t quads = (total + WPB - 1) / WPB;
  const int64_t per = (quads + gridDim.x - 1) / gridDim.x;
  const int64_t qbeg = (int64_t)blockIdx.x * per, qend = min(quads, qbeg + per);
  {
    for (int64_t qd = qbeg; qd < qend; ++qd) {
      const int64_t kb = qd * WPB;
      int sb = -1;
      int64_t base = 0;
      if (A.stage_bytes > 0) {
        const int2 f = A.blkmap[kb];
        const int t0 = A.op[f.x].type;
        const int32_t N0 = A.inst[f.x].N;
        const bool mine = (A.inst[f.x].prec32 != 0) == P32;
        const int64_t esz = P32 ? (int64_t)sizeof(float2) : (int64_t)sizeof(double2);
        if (mine && (t0 == BOP_TERM || t0 == BOP_POWACC) &&
            (int64_t)R * N0 * esz <= A.stage_bytes) {
          sb = f.x;
          const int64_t n0r = A.inst[f.x].n;
          base = ((int64_t)f.y * kWaveRows) / N0 * N0;
          __syncthreads();  // earlier blocks are done with xs
          if constexpr (P32)
            batch_stage<R>(reinterpret_cast<float2 *>(xs), A.op[f.x].x32, n0r, base, N0);
          else
            batch_stage<R>(xs, A.op[f.x].x, n0r, base, N0);
          __syncthreads();
        }
      }
      const int64_t g = kb + wave;  // wave-uniform
      if (g >= total) continue;
      const int2 bk = A.blkmap[g];
      const int b = bk.x;
      const BatchOp &O = A.op[b];
      const int type = O.type;
      if (type == BOP_NONE) continue;
      const BatchInst &I = A.inst[b];
      if ((I.prec32 != 0) != P32) continue;  // the other kernel's walk
      BatchSlots *S = &A.slots[b];
      const int64_t k = bk.y;
      const int64_t r0 = k * kWaveRows;
      const int64_t n = I.n;
      const int nr = (int)min((int64_t)kWaveRows, n - r0);
      const int64_t row = r0 + lane;
      const bool live = lane < nr;
      const double2 *ox = O.x;
      if constexpr (P32) {
      if (type == BOP_TERM) {
        SpmvArgs a{};
        a.n = n;
        a.rp = I.rp;
        a.wcol = I.wcol;
        a.wval32 = I.wval32;
        a.wcoef = I.wcoef;
        a.wcoef32 = I.wcoef32;
        a.wdiag32 = I.wdiag32;
        a.wstart = I.wstart;
        a.wshn = I.wshn;
        a.wshs = I.wshs;
        a.wsh = I.wsh;
        a.wsh_stride = I.wsh_stride;
        a.wlen = I.wlen;
        a.wperm = I.wperm;
        a.nwb = I.nwb;
        a.N = I.N;
        a.x32 = O.x32;
        BatchTerm32Epi<R> epi;
        epi.n = n;
        epi.alpha = O.alpha;
        epi.fin_hi = O.fin_hi;
        epi.fin_lo = O.fin_lo;
        epi.fout_hi = O.fout_hi;
        epi.fout_lo = O.fout_lo;
        epi.y = O.y32;
        epi.active = O.active;
        epi.first = O.first != 0;
  #pragma unroll
        for (int r = 0; r < R; ++r) epi.my[r] = epi.mf[r] = epi.mb0[r] = 0ull;
        const bool st = sb == b;
        const float2 *xs32 = reinterpret_cast<const float2 *>(xs);
        if (I.split)
          wave_block<R, true, true, BatchTerm32Epi<R>, true, true, true>(a, k, epi, xs32, base, st);
        else
          wave_block<R, true, true, BatchTerm32Epi<R>, true, false, true>(a, k, epi, xs32, base, st);
  #pragma unroll
        for (int r = 0; r < R; ++r) {
          batch_flush(epi.my[r], &S->y[r]);
          batch_flush(epi.mf[r], &S->f[r]);
          if (epi.first) batch_flush(epi.mb0[r], &S->b0[r]);
        }
      } else if (type == BOP_TRACE) {
        // one wave (the walk's first block) checks every column's trace
        if (k == 0) {
          for (int r = 0; r < R && r < I.n0; ++r) {
            const double tr = wave_trace(O.fout_hi + r * n, O.fout_lo + r * n, I.N);
            if (lane == 0) {
              if (!isfinite(tr)) *(volatile int *)A.nonfinite = 1;
              if (O.first) {
                S->tr0[r] = tr;
                S->scale[r] = 1.0;
              } else {
                // as trace32_kernel: scaled only when the deviation is small
                const double tr0 = S->tr0[r];
                const bool ok = isfinite(tr) && isfinite(tr0) && tr != 0.0 && tr0 != 0.0 &&
                                fabs(tr - tr0) <= 0x1p-10 * fabs(tr0);
                S->scale[r] = ok ? tr0 / tr : 1.0;
                const unsigned long long d = abs_bits(tr - tr0);
                if (d > S->trace_dev) S->trace_dev = d;
              }
            }
          }
        }
      } else if (type == BOP_LOAD) {
        // rho0 split into the state pair 0 (as split_c64_kernel); the other
        // vectors start at zero, so columns beyond n0 stay zero throughout
        if (live) {
          const int n0 = I.n0;
  #pragma unroll
          for (int r = 0; r < R; ++r) {
            const int64_t e = r * n + row;
            const double2 z = r < n0 ? gld(I.rho0 + e) : make_double2(0.0, 0.0);
            const float2 h = make_float2((float)z.x, (float)z.y);
            const float2 zf = make_float2(0.0f, 0.0f);
            gst(I.Ph[0] + e, h);
            gst(I.Pl[0] + e, make_float2((float)(z.x - (double)h.x), (float)(z.y - (double)h.y)));
            gst(I.Ph[1] + e, zf);
            gst(I.Pl[1] + e, zf);
            gst(I.B32[0] + e, zf);
            gst(I.B32[1] + e, zf);
          }
        }
      } else if (type == BOP_EMIT) {
        // (hi + lo) times the check's factor in complex128 (as emit32_kernel;
        // the pair re-split when the factor is not 1), or rho0 itself
        if (live) {
          const int64_t pt = O.point;
          const int N1 = I.N + 1;
          const int n0 = I.n0;
          double2 *out = I.out;
          double *pops = I.pops;
  #pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r >= n0) break;
            const int64_t e = r * n + row;
            double2 v;
            if (O.first) {
              v = gld(I.rho0 + e);
            } else {
              const double f = S->scale[r];
              const float2 h = gld(O.fout_hi + e), l = gld(O.fout_lo + e);
              v = make_double2(((double)h.x + (double)l.x) * f, ((double)h.y + (double)l.y) * f);
              if (f != 1.0) {
                const float2 h2 = make_float2((float)v.x, (float)v.y);
                gst(O.fout_hi + e, h2);
                gst(O.fout_lo + e,
                    make_float2((float)(v.x - (double)h2.x), (float)(v.y - (double)h2.y)));
              }
            }
            if (out) gst(out + (pt * n0 + r) * n + row, v);
            if (pops && row % N1 == 0) gst(pops + (pt * n0 + r) * I.N + row / N1, v.x);
          }
        }
      }
      } else {
      if (type == BOP_TERM || type == BOP_POWACC) {
        SpmvArgs a{};
        a.n = n;
        a.rp = I.rp;
        a.wcol = I.wcol;
        a.wval = I.wval;
        a.wval32 = I.wval32;
        a.wcoef = I.wcoef;
        a.wcoef32 = I.wcoef32;
        a.wdiag = I.wdiag;
        a.wdiag32 = I.wdiag32;
        a.wstart = I.wstart;
        a.wshn = I.wshn;
        a.wshs = I.wshs;
        a.wsh = I.wsh;
        a.wsh_stride = I.wsh_stride;
        a.wlen = I.wlen;
        a.wperm = I.wperm;
        a.nwb = I.nwb;
        a.N = I.N;
        a.x = ox;
        BatchTermEpi<R> epi;
        epi.n = n;
        epi.alpha = O.alpha;
        epi.kpow = O.kpow;
        epi.fin = O.fin;
        epi.fout = O.fout;
        epi.y = O.y;
        epi.active = O.active;
        epi.first = O.first != 0;
        epi.series = type == BOP_POWACC;
  #pragma unroll
        for (int r = 0; r < R; ++r) epi.my[r] = epi.mf[r] = epi.mb0[r] = 0ull;
        const bool st = sb == b;
        if (I.split) {
          if (I.f32)
            wave_block<R, true, true, BatchTermEpi<R>, true, true>(a, k, epi, xs, base, st);
          else
            wave_block<R, false, true, BatchTermEpi<R>, true, true>(a, k, epi, xs, base, st);
        } else if (I.f32) {
          wave_block<R, true, true, BatchTermEpi<R>, true>(a, k, epi, xs, base, st);
        } else {
          wave_block<R, false, true, BatchTermEpi<R>, true>(a, k, epi, xs, base, st);
        }
  #pragma unroll
        for (int r = 0; r < R; ++r) {
          batch_flush(epi.my[r], &S->y[r]);
          batch_flush(epi.mf[r], &S->f[r]);
          if (epi.first && !epi.series) batch_flush(epi.mb0[r], &S->b0[r]);
        }
      } else if (type == BOP_ACC) {
        const double2 *fin = O.fin;
        double2 *fout = O.fout;
        const double kpow = O.kpow;
        const uint32_t active = O.active;
        unsigned long long mf[R];
  #pragma unroll
        for (int r = 0; r < R; ++r) {
          mf[r] = 0ull;
          if (live && ((active >> r) & 1u)) {
            double2 f = gld(fin + r * n + row);
            const double2 kv = gld(ox + r * n + row);
            f.x = fma(kpow, kv.x, f.x);
            f.y = fma(kpow, kv.y, f.y);
            gst(fout + r * n + row, f);
            mf[r] = abs_bits(cabs2(f));
          }
        }
  #pragma unroll
        for (int r = 0; r < R; ++r) batch_flush(mf[r], &S->f[r]);
      } else if (type == BOP_NORM) {
  #pragma unroll
        for (int r = 0; r < R; ++r) {
          const unsigned long long m = live ? abs_bits(cabs2(gld(ox + r * n + row))) : 0ull;
          batch_flush(m, &S->b0[r]);
        }
      } else if (type == BOP_LOAD) {
        // rho0 into V[0]; every other work vector starts at zero, so columns
        // beyond n0 stay zero throughout
        if (live) {
          const double2 *rho0 = I.rho0;
          double2 *v0 = I.V[0], *v1 = I.V[1], *f0 = I.F[0], *f1 = I.F[1],
                  *b0 = I.B[0], *b1 = I.B[1];
          const int n0 = I.n0;
  #pragma unroll
          for (int r = 0; r < R; ++r) {
            const int64_t e = r * n + row;
            const double2 z = make_double2(0.0, 0.0);
            gst(v0 + e, r < n0 ? gld(rho0 + e) : z);
            gst(v1 + e, z);
            gst(f0 + e, z);
            gst(f1 + e, z);
            gst(b0 + e, z);
            gst(b1 + e, z);
          }
        }
      } else if (type == BOP_EMIT) {
        if (live) {
          const int64_t pt = O.point;
          const int N1 = I.N + 1;
          const int n0 = I.n0;
          double2 *out = I.out;
          double *pops = I.pops;
  #pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r >= n0) break;
            const double2 v = gld(ox + r * n + row);
            if (out) gst(out + (pt * n0 + r) * n + row, v);
            if (pops && row % N1 == 0) gst(pops + (pt * n0 + r) * I.N + row / N1, v.x);
          }
        }
      }
      }
    }
  }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_assemble(const AssembleArgs &a, int64_t n, hipStream_t s) {
  // one wave per 64-row block, grid-stride
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t want = (nwb + kBlock / 64 - 1) / (kBlock / 64);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_row_blocks(const int64_t *rp, int64_t n, int64_t B, int32_t *blk, int64_t nblk,
                             hipStream_t s) {
  hipLaunchKernelGGL(row_blocks_kernel, dim3(blocks_for(nblk + 1)), dim3(kBlock), 0, s, rp, n, B,
                     blk, nblk);
  return hipGetLastError();
}

hipError_t launch_wjag_plan(const int64_t *rp, const int32_t *col, const double2 *val, int64_t n,
                            int32_t N, bool shared, int32_t *wglob, int32_t *wshn, int64_t *wcnt,
                            hipStream_t s) {
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t grid = (nwb + kBlock / 64 - 1) / (kBlock / 64);
  if (shared)
    hipLaunchKernelGGL(wjag_plan_kernel<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, rp, col,
                       val, n, N, nwb, wglob, wshn, wcnt);
  else
    hipLaunchKernelGGL(wjag_plan_kernel<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, rp, col,
                       val, n, N, nwb, wglob, wshn, wcnt);
  return hipGetLastError();
}

hipError_t launch_wjag_fill(const int64_t *rp, const int32_t *col, const double2 *val, int64_t n,
                            int32_t N, bool split, const int32_t *wshn, const int64_t *wstart,
                            const int64_t *wshs, int32_t *wcol, double2 *wval, double *wcoef,
                            double2 *wdiag, int32_t *wlen, unsigned char *wperm, SharedEntry *wsh,
                            int *bad, hipStream_t s) {
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t grid = (nwb + kBlock / 64 - 1) / (kBlock / 64);
  if (split)
    hipLaunchKernelGGL(wjag_fill_kernel<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, rp, col,
                       val, n, N, nwb, wshn, wstart, wshs, wcol, wval, wcoef, wdiag, wlen, wperm,
                       wsh, bad);
  else
    hipLaunchKernelGGL(wjag_fill_kernel<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, rp, col,
                       val, n, N, nwb, wshn, wstart, wshs, wcol, wval, wcoef, wdiag, wlen, wperm,
                       wsh, bad);
  return hipGetLastError();
}

hipError_t launch_wjag_hash(const int32_t *wcol, const double *wcoef, const double2 *wval,
                            const int32_t *wlen, const int32_t *wshn, const int64_t *wstart,
                            int64_t n, unsigned long long *hash, hipStream_t s) {
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t grid = (nwb + kBlock / 64 - 1) / (kBlock / 64);
  hipLaunchKernelGGL(wjag_hash_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, wcol, wcoef, wval,
                     wlen, wshn, wstart, n, nwb, hash);
  return hipGetLastError();
}

hipError_t launch_wjag_same(const int32_t *wcol, const double *wcoef, const double2 *wval,
                            const int32_t *wlen, const int32_t *wshn, const int64_t *wstart,
                            int64_t n, const int64_t *canon, int *same, hipStream_t s) {
  const int64_t nwb = (n + kWaveRows - 1) / kWaveRows;
  const int64_t grid = (nwb + kBlock / 64 - 1) / (kBlock / 64);
  hipLaunchKernelGGL(wjag_same_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, wcol, wcoef, wval,
                     wlen, wshn, wstart, n, nwb, canon, same);
  return hipGetLastError();
}

hipError_t launch_row_abs_max(int64_t n, const int64_t *rp, const double2 *val,
                              unsigned long long *out_bits, hipStream_t s) {
  hipLaunchKernelGGL(row_abs_max_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, rp, val,
                     out_bits);
  return hipGetLastError();
}

hipError_t launch_adj_row_abs_max(int64_t n, int32_t N, const int64_t *rp, const double2 *val,
                                  const int64_t *frp, const int64_t *trp, const double *tval,
                                  unsigned long long *out_bits, hipStream_t s) {
  if (n <= 0 || N <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adj_row_abs_max_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, N, rp,
                     val, frp, trp, tval, out_bits);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  int grid = (int)((words + kBlock - 1) / kBlock);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(kBlock), 0, s, (unsigned int *)p, words);
  return hipGetLastError();
}

hipError_t launch_copy(double2 *dst, const double2 *src, int64_t n, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(float *dst, const double *src, int64_t n, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_to_c64(float2 *dst, const double2 *src, int64_t n, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(to_c64_kernel, dim3(grid), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

#define QSW_ENGINE_SWITCH(ENG, CALL)      \
  switch (ENG) {                          \
    case 0: CALL(0); break;               \
    case 1: CALL(1); break;               \
    case 10: CALL(10); break;             \
    case 11: CALL(11); break;             \
    case 100: CALL(100); break;           \
    case 101: CALL(101); break;           \
    case 110: CALL(110); break;           \
    case 111: CALL(111); break;           \
    case 200: CALL(200); break;           \
    case 201: CALL(201); break;           \
    case 210: CALL(210); break;           \
    case 211: CALL(211); break;           \
    case 300: CALL(300); break;           \
    case 310: CALL(310); break;           \
    case 3: CALL(3); break;               \
    case 4: CALL(4); break;               \
    case 8: CALL(8); break;               \
    case 16: CALL(16); break;             \
    case 32: CALL(32); break;             \
    case 64: CALL(64); break;             \
    default: return hipErrorInvalidValue; \
  }

// Dynamic LDS of a product launch: the staged rho-row for engines 1xx and
// 3xx, the rows of an XCD band for 2xx.
inline size_t stage_bytes(int engine, const SpmvArgs &a) {
  if (engine >= 200 && engine < 300) {
    const int bw = a.N / 64 / 8;
    return (size_t)(bw >= 4 ? 1 : 4 / bw) * a.N * sizeof(double2);
  }
  return engine >= 100 ? (size_t)a.N * sizeof(double2) : 0;
}

hipError_t launch_taylor_term(const SpmvArgs &a, int engine, int grid, hipStream_t s) {
#define QSW_L(E) \
  hipLaunchKernelGGL(term_kernel<E>, dim3(grid), dim3(kBlock), stage_bytes(E, a), s, a)
  QSW_ENGINE_SWITCH(engine, QSW_L)
#undef QSW_L
  return hipGetLastError();
}

hipError_t launch_taylor_term32(const SpmvArgs &a, int engine, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.N * sizeof(float2);
  switch (engine) {
    case 1: hipLaunchKernelGGL(term32_kernel<1>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 11: hipLaunchKernelGGL(term32_kernel<11>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 101: hipLaunchKernelGGL(term32_kernel<101>, dim3(grid), dim3(kBlock), lds, s, a); break;
    case 111: hipLaunchKernelGGL(term32_kernel<111>, dim3(grid), dim3(kBlock), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_split_c64(const double2 *v, float2 *hi, float2 *lo, int64_t n, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(split_c64_kernel, dim3(grid), dim3(kBlock), 0, s, v, hi, lo, n);
  return hipGetLastError();
}

hipError_t launch_trace32(DeviceState *st, const float2 *hi, const float2 *lo, int32_t N,
                          int reference, hipStream_t s) {
  hipLaunchKernelGGL(trace32_kernel, dim3(1), dim3(kBlock), 0, s, st, hi, lo, N, reference);
  return hipGetLastError();
}

hipError_t launch_emit32(const DeviceState *st, float2 *hi, float2 *lo, double2 *out, int64_t n,
                         hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(emit32_kernel, dim3(grid), dim3(kBlock), 0, s, st, hi, lo, out, n);
  return hipGetLastError();
}

hipError_t launch_spmv(const SpmvArgs &a, int engine, int grid, hipStream_t s) {
#define QSW_L(E) \
  hipLaunchKernelGGL(plain_kernel<E>, dim3(grid), dim3(kBlock), stage_bytes(E, a), s, a)
  QSW_ENGINE_SWITCH(engine, QSW_L)
#undef QSW_L
  return hipGetLastError();
}

hipError_t launch_series_init(DeviceState *st, PointSlots *pts, int npts, const double2 *Z,
                              int64_t n, int grid, hipStream_t s) {
  hipError_t e = launch_zero(&st->series, sizeof(SeriesSlots), s);
  if (e != hipSuccess) return e;
  e = launch_zero(pts, sizeof(PointSlots) * (size_t)npts, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(vec_norm_kernel, dim3(grid), dim3(kBlock), 0, s, Z, n, &st->series.kn[0]);
  return hipGetLastError();
}

hipError_t launch_series_power(const SpmvArgs &a, PointSlots *pt, int k, int p, int engine,
                               int grid, hipStream_t s) {
#define QSW_L(E) \
  hipLaunchKernelGGL(series_power_kernel<E>, dim3(grid), dim3(kBlock), stage_bytes(E, a), s, a, \
                     pt, k, p)
  QSW_ENGINE_SWITCH(engine, QSW_L)
#undef QSW_L
  return hipGetLastError();
}

hipError_t launch_series_accum(DeviceState *st, PointSlots *pt, int k, int p, const double2 *Kp,
                               const double2 *Z, double2 *F, int64_t n, double tol, int grid,
                               hipStream_t s) {
  hipLaunchKernelGGL(series_accum_kernel, dim3(grid), dim3(kBlock), 0, s, st, pt, k, p, Kp, Z, F,
                     n, tol);
  return hipGetLastError();
}

hipError_t launch_spmm2(const SpmvArgs &a, bool split, int mode, double *part, double2 *sgn,
                        double *h, int grid, hipStream_t s) {
  // both columns of the rho-row staged in LDS when they fit
  const size_t lds = (size_t)a.N * 2 * sizeof(double2);
  const bool stage = a.N > 0 && lds <= kStageMaxBytes;
#define QSW_L(SP, ST, AD, G, A)                                                           \
  hipLaunchKernelGGL((spmm2_kernel<SP, ST, AD>), dim3(G), dim3(kBlock), ST ? lds : 0, s, A, \
                     mode, part, sgn, h)
  if (a.adj_fwd) {
    // L^dagger through the phase-split layout of L: `grid` workgroups for
    // the blocks, then one wavefront per row (a, a)
    if (!split || !a.trp || mode == 1 || a.N < 1) return hipErrorInvalidValue;
    SpmvArgs b = a;
    b.adj_grid = grid;
    const int all = grid + (int)((a.N + kBlock / 64 - 1) / (kBlock / 64));
    if (stage) QSW_L(true, true, true, all, b);
    else QSW_L(true, false, true, all, b);
  } else if (split && stage) QSW_L(true, true, false, grid, a);
  else if (split) QSW_L(true, false, false, grid, a);
  else if (stage) QSW_L(false, true, false, grid, a);
  else QSW_L(false, false, false, grid, a);
#undef QSW_L
  return hipGetLastError();
}

hipError_t launch_spmm_wide(const SpmvArgs &a, bool split, int nr, const WideOut &o, int grid,
                            hipStream_t s) {
  if (nr < 2 || nr > 2 * kEstChainsMax || (nr & 1) || o.ys < 0 || o.ys > nr) return hipErrorInvalidValue;
  if (o.ys != nr - 2 * (o.fin ? 1 : 0)) return hipErrorInvalidValue;
  if (a.adj_fwd && (!split || !a.trp || (o.fin && o.mode == 1) || a.N < 1))
    return hipErrorInvalidValue;
  // ADJ: L^dagger through the phase-split layout of L: `grid` workgroups for
  // the blocks, then one wavefront per row (a, a)
  SpmvArgs b = a;
  b.adj_grid = grid;
  const int all = grid + (int)((a.N + kBlock / 64 - 1) / (kBlock / 64));
#define QSW_L(SP, R, AD, G, A) \
  hipLaunchKernelGGL((spmm_wide_kernel<SP, R, AD>), dim3(G), dim3(kBlock), 0, s, A, o)
#define QSW_W(R)                                \
  case R:                                       \
    if (a.adj_fwd) QSW_L(true, R, true, all, b); \
    else if (split) QSW_L(true, R, false, grid, a); \
    else QSW_L(false, R, false, grid, a);       \
    break;
  switch (nr) {
    QSW_W(2) QSW_W(4) QSW_W(6) QSW_W(8) QSW_W(10) QSW_W(12) QSW_W(14) QSW_W(16)
    default:
      return hipErrorInvalidValue;
  }
#undef QSW_W
#undef QSW_L
  return hipGetLastError();
}
static_assert(2 * kEstChainsMax == 16, "instantiated widths cover every chain count");

hipError_t launch_pack_pairs(double2 *W, int64_t n, const PairSources &ps, hipStream_t s) {
  if (ps.chains < 1 || ps.chains > kEstChainsMax) return hipErrorInvalidValue;
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(pack_pairs_kernel, dim3(grid), dim3(kBlock), 0, s, W, n, ps);
  return hipGetLastError();
}

hipError_t launch_unit_pairs(double2 *W, int64_t n, const PairUnits &pu, hipStream_t s) {
  if (pu.chains < 1 || pu.chains > kEstChainsMax) return hipErrorInvalidValue;
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(unit_pairs_kernel, dim3(grid), dim3(kBlock), 0, s, W, n, pu);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int nblocks, double *out2, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, part, nblocks, out2);
  return hipGetLastError();
}

// One wavefront: the small results, then the sequence number (a release
// store at system scope orders it after them for the host).
__global__ __launch_bounds__(64) void post_kernel(const double *v, int nv, const int64_t *iv,
                                                  int ni, const double *extra, HostPost *dst,
                                                  unsigned long long seq) {
  const int t = threadIdx.x;
  for (int q = t; q < nv; q += 64) dst->v[q] = v[q];
  for (int q = t; q < ni; q += 64) dst->i[q] = iv[q];
  if (t == 0 && extra) dst->v[nv] = *extra;
  __syncthreads();
  if (t == 0) __hip_atomic_store(&dst->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(64) void post_list_kernel(PostList l, HostPost *dst,
                                                       unsigned long long seq) {
  const int t = threadIdx.x;
  for (int j = 0; j < l.chains; ++j) {
    double *dv = dst->v + j * (kTopKMax + 1);
    int64_t *di = dst->i + j * kTopKMax;
    if (t < l.nv[j]) dv[t] = l.v[j][t];
    if (t < l.ni[j]) di[t] = l.i[j][t];
    if (t == 0 && l.extra[j]) dv[l.nv[j]] = *l.extra[j];
  }
  __syncthreads();
  if (t == 0) __hip_atomic_store(&dst->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_post_list(const PostList &l, HostPost *dst, unsigned long long seq,
                            hipStream_t s) {
  if (l.chains < 1 || l.chains > kEstChainsMax) return hipErrorInvalidValue;
  for (int j = 0; j < l.chains; ++j)
    if (l.nv[j] < 0 || l.ni[j] < 0 || l.nv[j] + 1 > kTopKMax + 1 || l.ni[j] > kTopKMax)
      return hipErrorInvalidValue;
  hipLaunchKernelGGL(post_list_kernel, dim3(1), dim3(64), 0, s, l, dst, seq);
  return hipGetLastError();
}

hipError_t launch_post(const double *v, int nv, const int64_t *iv, int ni, const double *extra,
                       HostPost *dst, unsigned long long seq, hipStream_t s) {
  if (nv < 0 || ni < 0 || nv + 1 > kPostMax || ni > kPostMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(post_kernel, dim3(1), dim3(64), 0, s, v, nv, iv, ni, extra, dst, seq);
  return hipGetLastError();
}

hipError_t launch_probe_init(double2 *X, int64_t n, int t, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(probe_init_kernel, dim3(grid), dim3(kBlock), 0, s, X, n, t);
  return hipGetLastError();
}

hipError_t launch_unit_cols(double2 *X, int64_t n, int64_t i0, int64_t i1, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(unit_cols_kernel, dim3(grid), dim3(kBlock), 0, s, X, n, i0, i1);
  return hipGetLastError();
}

hipError_t launch_swap_pairs(double2 *dst, const double2 *src, int64_t n, hipStream_t s) {
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(swap_pairs_kernel, dim3(grid), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_topk(const double *h, int64_t n, int K, int grid, double *cand_v, int64_t *cand_i,
                       double *out_v, int64_t *out_i, hipStream_t s) {
  if (K < 1 || K > kTopKMax) return hipErrorInvalidValue;
  // At most 256 partial workgroups: the one-workgroup merge scans every
  // candidate once per round (with 4096 partials it took 60 us).  The top K
  // under the (value, smaller index) order does not depend on the split.
  const int g = grid < 256 ? grid : 256;
  hipLaunchKernelGGL(topk_partial_kernel, dim3(g), dim3(kBlock), 0, s, h, n, K, cand_v, cand_i);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(topk_merge_kernel, dim3(1), dim3(kBlock), 0, s, cand_v, cand_i,
                     (int64_t)g * K, K, out_v, out_i);
  return hipGetLastError();
}

hipError_t launch_populations(const double2 *rho, int32_t N, int32_t count, double *pops,
                              hipStream_t s) {
  const int64_t total = (int64_t)N * count;
  hipLaunchKernelGGL(populations_kernel, dim3(blocks_for(total)), dim3(kBlock), 0, s, rho, N,
                     count, pops);
  return hipGetLastError();
}

hipError_t launch_batch_control(const BatchArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(batch_control_kernel, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_work(const BatchArgs &a, int rhs, bool p32, int grid, hipStream_t s) {
#define QSW_L(R)                                                                                  \
  if (p32)                                                                                        \
    hipLaunchKernelGGL((batch_work_kernel<R, true>), dim3(grid), dim3(kBlock), a.stage_bytes, s, a); \
  else                                                                                            \
    hipLaunchKernelGGL((batch_work_kernel<R, false>), dim3(grid), dim3(kBlock), a.stage_bytes, s, a);
  switch (rhs) {
    case 1: QSW_L(1) break;
    case 2: QSW_L(2) break;
    case 4: QSW_L(4) break;
    default: return hipErrorInvalidValue;
  }
#undef QSW_L
  return hipGetLastError();
}

hipError_t launch_batch_blocks(const BatchArgs &a, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  int grid = blocks_for(a.nblocks);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(batch_blocks_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int batch_resident_workgroups(int rhs) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e;
  if (rhs == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_work_kernel<1, false>, kBlock, 0);
  else if (rhs == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_work_kernel<2, false>, kBlock, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_work_kernel<4, false>, kBlock, 0);
  if (e != hipSuccess || per < 1) per = 1;
  return cus * per;
}

int resident_workgroups(int which) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e;
  if (which == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, spmm2_kernel<true, true>, kBlock,
                                                     kStageMaxBytes);
  else if (which == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, term_kernel<3>, kBlock, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, term_kernel<0>, kBlock, 0);
  if (e != hipSuccess || per < 1) per = 1;
  return cus * per;
}

}  // namespace qsw
