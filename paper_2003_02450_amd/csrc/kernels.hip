// HIP kernels of libqsw for gfx950 (MI355X): superoperator assembly, the
// complex128 CSR product with the fused Taylor-term epilogue, the
// time-series kernels and the block 1-norm estimation helpers.
//
// All maxima of non-negative doubles travel as IEEE bit patterns in 64-bit
// unsigned integers: their unsigned order is the numeric order, so a plain
// integer atomicMax merges them and the result does not depend on the order
// in which workgroups finish.  NaN (after fabs) sorts above +inf, so a
// non-finite value reaches the norm slots and is reported.
#include "qsw_impl.h"

#include <hip/hip_runtime.h>

namespace qsw {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

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

// Reduce NV maxima over the workgroup and merge them into dst[] with one
// atomic per value.  Every thread of the workgroup must call it.
// A maximum at or above the bit pattern of +inf flags *nonfinite.
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

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

// Streaming load of a matrix value: read once per product, so it is marked
// non-temporal to leave the caches to the gathered vector.
__device__ __forceinline__ double2 load_stream(const double2 *p) {
  const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(p));
  return make_double2(v.x, v.y);
}

// Complex multiply-accumulate acc += v * x.
__device__ __forceinline__ void cmac(double &ax, double &ay, double2 v, double2 x) {
  ax = fma(v.x, x.x, ax);
  ax = fma(-v.y, x.y, ax);
  ay = fma(v.x, x.y, ay);
  ay = fma(v.y, x.x, ay);
}

// Row product of LPR lanes: lanes stride through the row, then a butterfly
// over the LPR lanes leaves the full sum in every lane of the group.
template <int LPR>
__device__ __forceinline__ double2 row_dot(const int64_t *__restrict__ rp,
                                           const int32_t *__restrict__ col,
                                           const double2 *__restrict__ val,
                                           const double2 *__restrict__ x, int64_t row,
                                           bool valid, int lane) {
  double ax = 0.0, ay = 0.0;
  if (valid) {
    const int64_t e0 = rp[row], e1 = rp[row + 1];
    for (int64_t e = e0 + lane; e < e1; e += LPR) {
      const int c = __builtin_nontemporal_load(col + e);
      const double2 v = load_stream(val + e);
      cmac(ax, ay, v, x[c]);
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
    ax += __shfl_xor(ax, off, LPR);
    ay += __shfl_xor(ay, off, LPR);
  }
  return make_double2(ax, ay);
}

// --------------------------------------------------------------------------
// Superoperator assembly: one thread per row r = a*N + b.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void assemble_kernel(AssembleArgs A, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int64_t N = A.N;
  const int64_t a = r / N, b = r - a * N;
  const int64_t ha0 = A.hp[a], ha1 = A.hp[a + 1];
  const int64_t hb0 = A.hp[b], hb1 = A.hp[b + 1];
  const int64_t degHa = ha1 - ha0;
  const int64_t ra0 = A.rp[a], ra1 = A.rp[a + 1];
  const int64_t degRa = ra1 - ra0;
  // Rows before (a, 0): sum over a' < a of (N degH(a') + E_H + N + degR(a'));
  // rows (a, b') with b' < b: b' (degH(a) + 1) + degH(b') plus the
  // population-transfer entries of row (a, a) once b > a.
  const int64_t start = N * A.PH[a] + a * (A.EH + N) + A.PR[a] + b * (degHa + 1) + A.PH[b] +
                        (b > a ? degRa : 0);
  A.row_ptr[r] = start;
  if (r == n - 1) A.row_ptr[n] = 2 * N * A.EH + N * N + A.PR[N];

  const double ch = A.sigma * (1.0 - A.omega);  // sigma (1 - omega)
  const double w = A.omega;
  // diagonal: sigma(-i)(1-w)(H_aa - H_bb) - w/2 (K_a + K_b) + [a==b] w R_aa
  const double2 dval =
      make_double2(-0.5 * w * (A.K[a] + A.K[b]) + (a == b ? w * A.rdiag[a] : 0.0),
                   -ch * (A.hdiag[a] - A.hdiag[b]));
  const int64_t INF = INT64_MAX;
  int64_t i1 = ha0, i2 = hb0;
  int64_t i3 = (a == b) ? ra0 : 0, e3 = (a == b) ? ra1 : 0;
  bool diag_done = false;
  int64_t o = start;
  for (;;) {
    // S1: rho_cb terms, column c N + b, value sigma(-i)(1-w) H_ac
    const int64_t k1 = i1 < ha1 ? (int64_t)A.hc[i1] * N + b : INF;
    // S2: rho_ac terms, column a N + c, value sigma(+i)(1-w) conj(H_bc), and the diagonal
    const int64_t kh = i2 < hb1 ? a * N + A.hc[i2] : INF;
    const int64_t kd = diag_done ? INF : a * N + b;
    const int64_t k2 = kh < kd ? kh : kd;
    // S3: population transfer rho_jj, column j (N + 1), value w R_aj
    const int64_t k3 = i3 < e3 ? (int64_t)A.rc[i3] * (N + 1) : INF;
    if (k1 == INF && k2 == INF && k3 == INF) break;
    int64_t key;
    double2 v;
    if (k1 < k2 && k1 < k3) {
      const double2 h = A.hv[i1++];
      key = k1;
      v = make_double2(ch * h.y, -ch * h.x);
    } else if (k2 < k3) {
      key = k2;
      if (kd < kh) {
        v = dval;
        diag_done = true;
      } else {
        const double2 h = A.hv[i2++];
        v = make_double2(ch * h.y, ch * h.x);
      }
    } else {
      key = k3;
      v = make_double2(w * A.rv[i3++], 0.0);
    }
    A.col[o] = (int32_t)key;
    A.val[o] = v;
    ++o;
  }
}

// max over rows of sum_e |val[e]|  (on the adjoint this is ||L||_1).
__global__ __launch_bounds__(kBlock) void row_abs_max_kernel(int64_t n, const int64_t *rp,
                                                             const double2 *val,
                                                             unsigned long long *out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long m[1] = {0ull};
  if (r < n) {
    double s = 0.0;
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) s += cabs2(val[e]);
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

__global__ void copy_kernel(double2 *dst, const double2 *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// --------------------------------------------------------------------------
// Term j of one scaling step of the single-time algorithm.
// --------------------------------------------------------------------------
template <int LPR, bool TAYLOR>
__global__ __launch_bounds__(kBlock) void term_kernel(SpmvArgs a) {
  StepSlots *S = nullptr;
  if (TAYLOR) {
    S = &a.st->step[a.par];
    if (a.j >= 2) {
      if (*(volatile int *)&S->stop) return;
      const double c1 = bits_to_d(a.j == 2 ? S->b0 : S->b[a.j - 2]);
      const double c2 = bits_to_d(S->b[a.j - 1]);
      const double f = bits_to_d(S->f[a.j - 1]);
      if (c1 + c2 <= a.tol * f) {
        if (threadIdx.x == 0) *(volatile int *)&S->stop = 1;
        return;
      }
    } else if (blockIdx.x == 0) {
      // first term of a step: clear the other parity for the next step
      unsigned int *o = (unsigned int *)&a.st->step[a.par ^ 1];
      for (int i = threadIdx.x; i < (int)(sizeof(StepSlots) / 4); i += kBlock) o[i] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.st->products, 1ull);
  }
  constexpr int RPI = kBlock / LPR;
  const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t r1 = min(a.n, r0 + a.rows_per_block);
  unsigned long long mb = 0, mf = 0, mb0 = 0;
  for (int64_t base = r0; base < r1; base += RPI) {
    const int64_t row = base + g;
    const bool valid = row < r1;
    const double2 acc = row_dot<LPR>(a.rp, a.col, a.val, a.x, row, valid, lane);
    if (valid && lane == 0) {
      const double2 y = make_double2(a.alpha * acc.x, a.alpha * acc.y);
      a.y[row] = y;
      if (TAYLOR) {
        double2 f = a.fin[row];
        if (a.j == 1) mb0 = umax(mb0, abs_bits(cabs2(f)));
        f.x += y.x;
        f.y += y.y;
        a.fout[row] = f;
        mb = umax(mb, abs_bits(cabs2(y)));
        mf = umax(mf, abs_bits(cabs2(f)));
      }
    }
  }
  if (TAYLOR) {
    unsigned long long v[3] = {mb, mf, mb0};
    unsigned long long *const dst[3] = {&S->b[a.j], &S->f[a.j], a.j == 1 ? &S->b0 : nullptr};
    block_umax_to<3>(v, dst, &a.st->nonfinite);
  }
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
  if (*(volatile int *)&pt->stop) return true;
  if (p < 2) return false;
  const int q = p - 1;  // last term added
  const double kk = (double)k;
  const double c1 = (q == 1) ? bits_to_d(st->series.kn[0])
                             : pow(kk, (double)(q - 1)) * bits_to_d(st->series.kn[q - 1]);
  const double c2 = pow(kk, (double)q) * bits_to_d(st->series.kn[q]);
  if (c1 + c2 <= tol * bits_to_d(pt->f[q])) {
    if (threadIdx.x == 0) *(volatile int *)&pt->stop = 1;
    return true;
  }
  return false;
}

template <int LPR>
__global__ __launch_bounds__(kBlock) void series_power_kernel(SpmvArgs a, PointSlots *pt, int k,
                                                              int p) {
  if (point_done(a.st, pt, k, p, a.tol)) return;
  if (p <= *(volatile int *)&a.st->series.mhat) return;  // K_p already formed
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.st->products, 1ull);
  constexpr int RPI = kBlock / LPR;
  const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t r1 = min(a.n, r0 + a.rows_per_block);
  unsigned long long mk = 0;
  for (int64_t base = r0; base < r1; base += RPI) {
    const int64_t row = base + g;
    const bool valid = row < r1;
    const double2 acc = row_dot<LPR>(a.rp, a.col, a.val, a.x, row, valid, lane);
    if (valid && lane == 0) {
      const double2 y = make_double2(a.alpha * acc.x, a.alpha * acc.y);
      a.y[row] = y;
      mk = umax(mk, abs_bits(cabs2(y)));
    }
  }
  unsigned long long v[1] = {mk};
  unsigned long long *const dst[1] = {&a.st->series.kn[p]};
  block_umax_to<1>(v, dst, &a.st->nonfinite);
}

__global__ __launch_bounds__(kBlock) void series_accum_kernel(DeviceState *st, PointSlots *pt,
                                                              int k, int p, const double2 *Kp,
                                                              const double2 *Z, double2 *F,
                                                              int64_t n, double tol) {
  if (*(volatile int *)&pt->stop) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&st->series.mhat, p);
  const double kp = pow((double)k, (double)p);
  unsigned long long mf = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double2 kv = Kp[i];
    double2 f = (p == 1) ? Z[i] : F[i];
    f.x = fma(kp, kv.x, f.x);
    f.y = fma(kp, kv.y, f.y);
    F[i] = f;
    mf = umax(mf, abs_bits(cabs2(f)));
  }
  unsigned long long v[1] = {mf};
  unsigned long long *const dst[1] = {&pt->f[p]};
  block_umax_to<1>(v, dst, &st->nonfinite);
}

// --------------------------------------------------------------------------
// Two right-hand sides (block 1-norm estimation).
// --------------------------------------------------------------------------
template <int LPR>
__global__ __launch_bounds__(kBlock) void spmm2_kernel(int64_t n, const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const double2 *__restrict__ val,
                                                       const double2 *__restrict__ X,
                                                       double2 *__restrict__ Y, int mode,
                                                       double *part, double2 *sgn, double *h,
                                                       int64_t rows_per_block) {
  constexpr int RPI = kBlock / LPR;
  const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t base = r0; base < r1; base += RPI) {
    const int64_t row = base + g;
    double a0x = 0, a0y = 0, a1x = 0, a1y = 0;
    if (row < r1) {
      for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += LPR) {
        const int c = col[e];
        const double2 v = val[e];
        cmac(a0x, a0y, v, X[2 * (int64_t)c]);
        cmac(a1x, a1y, v, X[2 * (int64_t)c + 1]);
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      a0x += __shfl_xor(a0x, off, LPR);
      a0y += __shfl_xor(a0y, off, LPR);
      a1x += __shfl_xor(a1x, off, LPR);
      a1y += __shfl_xor(a1y, off, LPR);
    }
    if (row < r1 && lane == 0) {
      const double2 y0 = make_double2(a0x, a0y), y1 = make_double2(a1x, a1y);
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
  }
  if (mode == 1) {
    // deterministic per-block column sums: fixed tree over the workgroup
    __shared__ double sm0[kBlock], sm1[kBlock];
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
      part[2 * blockIdx.x] = sm0[0];
      part[2 * blockIdx.x + 1] = sm1[0];
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

template <int LPR>
hipError_t term_dispatch(const SpmvArgs &a, int grid, hipStream_t s, bool taylor) {
  if (taylor)
    hipLaunchKernelGGL((term_kernel<LPR, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((term_kernel<LPR, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_assemble(const AssembleArgs &a, int64_t n, hipStream_t s) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_row_abs_max(int64_t n, const int64_t *rp, const double2 *val,
                              unsigned long long *out_bits, hipStream_t s) {
  hipLaunchKernelGGL(row_abs_max_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, rp, val,
                     out_bits);
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

hipError_t launch_taylor_term(const SpmvArgs &a, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 4: return term_dispatch<4>(a, grid, s, true);
    case 8: return term_dispatch<8>(a, grid, s, true);
    case 16: return term_dispatch<16>(a, grid, s, true);
    case 32: return term_dispatch<32>(a, grid, s, true);
    case 64: return term_dispatch<64>(a, grid, s, true);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spmv(const SpmvArgs &a, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 4: return term_dispatch<4>(a, grid, s, false);
    case 8: return term_dispatch<8>(a, grid, s, false);
    case 16: return term_dispatch<16>(a, grid, s, false);
    case 32: return term_dispatch<32>(a, grid, s, false);
    case 64: return term_dispatch<64>(a, grid, s, false);
    default: return hipErrorInvalidValue;
  }
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

hipError_t launch_series_power(const SpmvArgs &a, PointSlots *pt, int k, int p, int lpr,
                               int grid, hipStream_t s) {
  switch (lpr) {
    case 4:
      hipLaunchKernelGGL(series_power_kernel<4>, dim3(grid), dim3(kBlock), 0, s, a, pt, k, p);
      break;
    case 8:
      hipLaunchKernelGGL(series_power_kernel<8>, dim3(grid), dim3(kBlock), 0, s, a, pt, k, p);
      break;
    case 16:
      hipLaunchKernelGGL(series_power_kernel<16>, dim3(grid), dim3(kBlock), 0, s, a, pt, k, p);
      break;
    case 32:
      hipLaunchKernelGGL(series_power_kernel<32>, dim3(grid), dim3(kBlock), 0, s, a, pt, k, p);
      break;
    case 64:
      hipLaunchKernelGGL(series_power_kernel<64>, dim3(grid), dim3(kBlock), 0, s, a, pt, k, p);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_series_accum(DeviceState *st, PointSlots *pt, int k, int p, const double2 *Kp,
                               const double2 *Z, double2 *F, int64_t n, double tol, int grid,
                               hipStream_t s) {
  hipLaunchKernelGGL(series_accum_kernel, dim3(grid), dim3(kBlock), 0, s, st, pt, k, p, Kp, Z, F,
                     n, tol);
  return hipGetLastError();
}

int spmm2_blocks(int64_t n, int grid) {
  constexpr int RPI = kBlock / 8;
  int64_t rpb = (n + grid - 1) / grid;
  rpb = (rpb + RPI - 1) / RPI * RPI;
  return (int)((n + rpb - 1) / rpb);
}

hipError_t launch_spmm2(int64_t n, const int64_t *rp, const int32_t *col, const double2 *val,
                        const double2 *X, double2 *Y, int mode, double *part, double2 *sgn,
                        double *h, int grid, hipStream_t s) {
  constexpr int LPR = 8;
  constexpr int RPI = kBlock / LPR;
  int64_t rpb = (n + grid - 1) / grid;
  rpb = (rpb + RPI - 1) / RPI * RPI;
  const int g = (int)((n + rpb - 1) / rpb);
  hipLaunchKernelGGL(spmm2_kernel<LPR>, dim3(g), dim3(kBlock), 0, s, n, rp, col, val, X, Y, mode,
                     part, sgn, h, rpb);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int nblocks, double *out2, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, part, nblocks, out2);
  return hipGetLastError();
}

hipError_t launch_populations(const double2 *rho, int32_t N, int32_t count, double *pops,
                              hipStream_t s) {
  const int64_t total = (int64_t)N * count;
  hipLaunchKernelGGL(populations_kernel, dim3(blocks_for(total)), dim3(kBlock), 0, s, rho, N,
                     count, pops);
  return hipGetLastError();
}

}  // namespace qsw
