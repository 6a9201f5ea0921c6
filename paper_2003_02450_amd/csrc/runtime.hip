// Host runtime and C ABI of libqsw (declared in include/qsw.h).
//
// Build: graph -> H, rates R, K on the host (O(N + E)), device assembly of
// the superoperator L and of its adjoint, exact ||L||_1 from the adjoint's
// row sums, block 1-norm estimates of ||L^p||_1 (p = 2..9), adjoint freed.
// Propagate: FP64 parameter selection on the host, then launch chains of the
// fused Taylor-term kernel whose stopping test runs on the device, so the
// host never waits inside the loop.
#include "handle.h"
#include "params.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <complex>
#include <limits>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <new>
#include <vector>

using namespace qsw;

namespace {

// Host-side operator data before upload.
struct HostOps {
  int32_t N = 0;
  std::vector<int64_t> hp;      // off-diagonal H CSR
  std::vector<int32_t> hc;
  std::vector<double> hv;       // interleaved complex
  std::vector<double> hdiag;
  std::vector<int64_t> rp;      // off-diagonal rates CSR (row = target)
  std::vector<int32_t> rc;
  std::vector<double> rv;
  std::vector<double> rdiag;
  // rates outside omega (absorption / emission channels), same layout; empty
  // when there are none
  std::vector<int64_t> fp;
  std::vector<int32_t> fc;
  std::vector<double> fv;
  std::vector<double> fdiag;
};

// The rates the assembly uses: omega R + F when there are rates outside
// omega (then pre-scaled: factor 1), else R itself with factor omega.
struct Rates {
  std::vector<int64_t> rp;
  std::vector<int32_t> rc;
  std::vector<double> rv;
  std::vector<double> rdiag;
  double scale = 1.0;
};

Rates effective_rates(const HostOps &op, double omega) {
  Rates R;
  const int32_t N = op.N;
  if (op.fp.empty()) {
    R.rp = op.rp;
    R.rc = op.rc;
    R.rv = op.rv;
    R.rdiag = op.rdiag;
    R.scale = omega;
    return R;
  }
  R.rp.assign(N + 1, 0);
  R.rdiag.assign(N, 0.0);
  for (int32_t i = 0; i < N; ++i) {
    int64_t a = op.rp[i], b = op.fp[i];
    while (a < op.rp[i + 1] || b < op.fp[i + 1]) {
      const int32_t ca = a < op.rp[i + 1] ? op.rc[a] : INT32_MAX;
      const int32_t cb = b < op.fp[i + 1] ? op.fc[b] : INT32_MAX;
      if (ca == cb) {
        R.rc.push_back(ca);
        R.rv.push_back(omega * op.rv[a++] + op.fv[b++]);
      } else if (ca < cb) {
        R.rc.push_back(ca);
        R.rv.push_back(omega * op.rv[a++]);
      } else {
        R.rc.push_back(cb);
        R.rv.push_back(op.fv[b++]);
      }
    }
    R.rp[i + 1] = (int64_t)R.rc.size();
    R.rdiag[i] = omega * op.rdiag[i] + (op.fdiag.empty() ? 0.0 : op.fdiag[i]);
  }
  R.scale = 1.0;
  return R;
}

// Check a host CSR: row_ptr monotone from 0, columns in range, strictly
// increasing within each row.
qsw_status_t check_csr(int32_t N, const int64_t *rp, const int32_t *ci, bool allow_diag) {
  if (rp[0] != 0) return QSW_ERR_GRAPH;
  for (int32_t i = 0; i < N; ++i) {
    if (rp[i + 1] < rp[i]) return QSW_ERR_GRAPH;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t c = ci[e];
      if (c < 0 || c >= N) return QSW_ERR_GRAPH;
      if (!allow_diag && c == i) return QSW_ERR_GRAPH;
      if (e > rp[i] && ci[e - 1] >= c) return QSW_ERR_GRAPH;
    }
  }
  return QSW_OK;
}

// Transpose of an N x N CSR (row-sorted output).
void transpose_csr(int32_t N, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, int width, std::vector<int64_t> &tp,
                   std::vector<int32_t> &tc, std::vector<double> &tv) {
  const int64_t nnz = rp[N];
  tp.assign(N + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) tp[ci[e] + 1]++;
  for (int32_t i = 0; i < N; ++i) tp[i + 1] += tp[i];
  tc.resize(nnz);
  tv.resize(nnz * width);
  std::vector<int64_t> pos(tp.begin(), tp.end() - 1);
  for (int32_t i = 0; i < N; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t o = pos[ci[e]]++;
      tc[o] = i;
      for (int w = 0; w < width; ++w) tv[o * width + w] = v[e * width + w];
    }
}

}  // namespace

namespace {

// Row blocks of the stream engine for one CSR: block budget B entries so that
// a block (whose rows start before the next multiple of B) never exceeds the
// LDS stage of `cap` entries when the longest row is at most cap/2.  The
// workgroups, a multiple of 8 so that runs of blocks map to one XCD each,
// take equal runs of blocks in at most two rounds of the stream kernel's own
// resident workgroups (`resident`; QSW_CSR_GRID overrides the two rounds).
// Rounds that end part-full leave a tail: on the 1024-vertex operator (21808
// blocks, 1024 resident) a product took 295 us at 992 workgroups, 291 at
// 1984, 365 at 1456, 328 at 1680, 333 at 2424 and 305-309 at 2728-7272.
struct Layout {
  int32_t *blk = nullptr;
  int32_t nblk = 0;
  int32_t bpw = 0;
  int grid = 0;
};

hipError_t make_layout(const int64_t *rp, int64_t n, int64_t nnz, int64_t maxrow, int cap,
                       int resident, hipStream_t s, Layout &L) {
  const int64_t B = (maxrow <= cap / 2) ? cap - maxrow : cap / 2;
  const int64_t nblk = std::max<int64_t>(1, (nnz + B - 1) / B);
  hipError_t e = dalloc(&L.blk, (size_t)nblk + 1);
  if (e != hipSuccess) return e;
  e = launch_row_blocks(rp, n, B, L.blk, nblk, s);
  if (e != hipSuccess) return e;
  int64_t G = std::max(8, 2 * resident / 8 * 8);
  G = std::min<int64_t>(G, env_int("QSW_GRID", (int)G));
  G = std::max(1, env_int("QSW_CSR_GRID", (int)G));
  if (G > nblk) G = nblk;
  if (G < 1) G = 1;
  const int64_t bpw = (nblk + G - 1) / G;
  int64_t g2 = (nblk + bpw - 1) / bpw;
  if (g2 >= 8) g2 = (g2 + 7) / 8 * 8;
  L.nblk = (int32_t)nblk;
  L.bpw = (int32_t)bpw;
  L.grid = (int)g2;
  return hipSuccess;
}

void choose_vector_launch(qsw_superop_s *h, int lpr) {
  const int rpi = kBlockThreads / lpr;
  const int target = 2048;
  int64_t rpb = (h->n + target - 1) / target;
  rpb = std::max<int64_t>(rpi, (rpb + rpi - 1) / rpi * rpi);
  h->engine = lpr;
  h->rows_per_block = rpb;
  h->grid = (int)((h->n + rpb - 1) / rpb);
}

// Upper bound of the longest row of L and of its adjoint: row (a, b) holds
// deg_H(a) + deg_H(b) + 1 entries, plus the population-transfer entries when
// a == b (rates of row a, or of column a for the adjoint).
int64_t max_row_bound(const HostOps &op, const Rates &R) {
  int64_t dh = 0, dr = 0;
  std::vector<int64_t> indeg(op.N, 0);
  for (int32_t i = 0; i < op.N; ++i) {
    dh = std::max<int64_t>(dh, op.hp[i + 1] - op.hp[i]);
    dr = std::max<int64_t>(dr, R.rp[i + 1] - R.rp[i]);
    for (int64_t e = R.rp[i]; e < R.rp[i + 1]; ++e) indeg[R.rc[e]]++;
  }
  for (int32_t i = 0; i < op.N; ++i) dr = std::max(dr, indeg[i]);
  return 2 * dh + 1 + dr;
}

// Device copies of one operator set plus the assembled matrix.
struct DeviceOps {
  int64_t *hp = nullptr;
  int32_t *hc = nullptr;
  double2 *hv = nullptr;
  double *hdiag = nullptr;
  int64_t *rp = nullptr;
  int32_t *rc = nullptr;
  double *rv = nullptr;
  double *rdiag = nullptr;
  double *K = nullptr;
  int64_t *PH = nullptr;
  int64_t *PR = nullptr;
  char *block = nullptr;  // all of the above, one allocation
  void release() { dfree(block); }
};

// Host arrays uploaded as one device block: one allocation and one copy
// (eleven pageable copies took about 40 us each).  Each array starts on a
// 256-byte boundary.  The staging vector must outlive the copy.
struct PackedUpload {
  struct Item {
    void **dst;
    const void *src;
    size_t bytes;
  };
  std::vector<Item> items;
  std::vector<char> host;
  template <class T>
  void add(T **dst, const void *src, size_t count) {
    items.push_back({(void **)dst, src, count * sizeof(T)});
  }
  hipError_t run(char **block, hipStream_t s) {
    std::vector<size_t> off;
    size_t total = 0;
    for (const Item &it : items) {
      off.push_back(total);
      total += (it.bytes + 255) & ~(size_t)255;
    }
    if (total == 0) total = 256;
    hipError_t e = dalloc(block, total);
    if (e != hipSuccess) return e;
    host.assign(total, 0);
    for (size_t k = 0; k < items.size(); ++k) {
      if (items[k].bytes) std::memcpy(host.data() + off[k], items[k].src, items[k].bytes);
      *items[k].dst = *block + off[k];
    }
    return hipMemcpyAsync(*block, host.data(), total, hipMemcpyHostToDevice, s);
  }
};

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src, hipStream_t s) {
  hipError_t e = dalloc(dst, src.size());
  if (e != hipSuccess) return e;
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Assemble sigma = +1 (L, rates as given) or -1 (L^dagger, rates transposed)
// into freshly allocated (row_ptr, col, val).
qsw_status_t assemble(const HostOps &op, const Rates &R, bool adjoint, double omega,
                      hipStream_t s, int64_t **rp_out, int32_t **col_out, double2 **val_out,
                      int64_t *nnz_out) {
  const int32_t N = op.N;
  const int64_t n = (int64_t)N * N;
  std::vector<int64_t> rtp;
  std::vector<int32_t> rtc;
  std::vector<double> rtv;
  const std::vector<int64_t> *rp = &R.rp;
  const std::vector<int32_t> *rc = &R.rc;
  const std::vector<double> *rv = &R.rv;
  if (adjoint) {
    transpose_csr(N, R.rp, R.rc, R.rv, 1, rtp, rtc, rtv);
    rp = &rtp;
    rc = &rtc;
    rv = &rtv;
  }
  // K_j = sum_i R_ij over the rates (diagonal included), for L and L^dagger
  std::vector<double> K(N, 0.0);
  for (int32_t i = 0; i < N; ++i) {
    for (int64_t e = R.rp[i]; e < R.rp[i + 1]; ++e) K[R.rc[e]] += R.rv[e];
    K[i] += R.rdiag[i];
  }
  std::vector<int64_t> PH(N + 1, 0), PR(N + 1, 0);
  for (int32_t i = 0; i < N; ++i) {
    PH[i + 1] = PH[i] + (op.hp[i + 1] - op.hp[i]);
    PR[i + 1] = PR[i] + ((*rp)[i + 1] - (*rp)[i]);
  }
  const int64_t EH = PH[N];
  const int64_t nnz = 2 * (int64_t)N * EH + n + PR[N];
  DeviceOps d;
  std::vector<double> hvec = op.hv;
  qsw_status_t st = QSW_OK;
  hipError_t e;
  int64_t *drp = nullptr;
  int32_t *dcol = nullptr;
  double2 *dval = nullptr;
  PackedUpload up;
  do {
    up.add<int64_t>(&d.hp, op.hp.data(), op.hp.size());
    up.add<int32_t>(&d.hc, op.hc.data(), op.hc.size());
    up.add<double2>(&d.hv, hvec.data(), hvec.size() / 2);
    up.add<double>(&d.hdiag, op.hdiag.data(), op.hdiag.size());
    up.add<int64_t>(&d.rp, rp->data(), rp->size());
    up.add<int32_t>(&d.rc, rc->data(), rc->size());
    up.add<double>(&d.rv, rv->data(), rv->size());
    up.add<double>(&d.rdiag, R.rdiag.data(), R.rdiag.size());
    up.add<double>(&d.K, K.data(), K.size());
    up.add<int64_t>(&d.PH, PH.data(), PH.size());
    up.add<int64_t>(&d.PR, PR.data(), PR.size());
    if ((e = up.run(&d.block, s)) != hipSuccess) break;
    if ((e = dalloc(&drp, (size_t)n + 1)) != hipSuccess) break;
    if ((e = dalloc(&dcol, (size_t)nnz)) != hipSuccess) break;
    if ((e = dalloc(&dval, (size_t)nnz)) != hipSuccess) break;
    AssembleArgs A;
    A.N = N;
    A.hp = d.hp; A.hc = d.hc; A.hv = d.hv; A.hdiag = d.hdiag;
    A.rp = d.rp; A.rc = d.rc; A.rv = d.rv; A.rdiag = d.rdiag;
    A.K = d.K; A.PH = d.PH; A.PR = d.PR; A.EH = EH;
    A.omega = omega;
    A.rscale = R.scale;
    A.sigma = adjoint ? -1.0 : 1.0;
    A.row_ptr = drp; A.col = dcol; A.val = dval;
    if ((e = launch_assemble(A, n, s)) != hipSuccess) break;
    e = hipStreamSynchronize(s);  // host vectors above must outlive the copies
  } while (false);
  d.release();
  if (e != hipSuccess) {
    dfree(drp); dfree(dcol); dfree(dval);
    st = status_of(e);
    return st;
  }
  *rp_out = drp;
  *col_out = dcol;
  *val_out = dval;
  *nnz_out = nnz;
  return QSW_OK;
}

// Block 1-norm estimator (Higham and Tisseur's algorithm, two columns,
// complex case, at most five iterations) applied to A^p, with the products
// formed by p sparse products on the device and the ranking of the
// candidate columns done on the device; the host reads back a few scalars
// per iteration.  Returns the estimate and the unit column (or probe column)
// that attains it.
// Pinned mailboxes (HostPost) of finished builds, kept per device for later
// builds (a pinned allocation costs more than a build's waits save).
struct PostPool {
  std::mutex mu;
  std::map<int, std::vector<std::pair<HostPost *, HostPost *>>> free;  // device -> (host, dev)
};
PostPool &post_pool() {
  static PostPool *p = new PostPool();  // kept until the process ends
  return *p;
}
hipError_t post_get(HostPost **host, HostPost **dev) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  PostPool &P = post_pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto &v = P.free[d];
    if (!v.empty()) {
      *host = v.back().first;
      *dev = v.back().second;
      v.pop_back();
      return hipSuccess;
    }
  }
  void *hp = nullptr, *dp = nullptr;
  if ((e = hipHostMalloc(&hp, sizeof(HostPost), hipHostMallocCoherent)) != hipSuccess) return e;
  if ((e = hipHostGetDevicePointer(&dp, hp, 0)) != hipSuccess) {
    (void)hipHostFree(hp);
    return e;
  }
  std::memset(hp, 0, sizeof(HostPost));
  *host = (HostPost *)hp;
  *dev = (HostPost *)dp;
  return hipSuccess;
}
void post_put(HostPost *host, HostPost *dev) {
  if (!host) return;
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return;
  PostPool &P = post_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  P.free[d].push_back({host, dev});
}

struct Estimator {
  int64_t n;
  hipStream_t s;
  SpmvArgs fwd{}, adj{};          // A and A^dagger (jagged layouts)
  bool fsplit = false, asplit = false;  // their value formats
  int grid = 0;                   // workgroups of a product (= partial sums per column)
  double2 *X, *Y, *W0, *W1, *S;  // n x 2 interleaved blocks
  double *h, *part, *sums;
  double *cand_v, *top_v;
  int64_t *cand_i, *top_i;
  int products = 0;
  // first iteration of every estimate, from one chain of products (first_pass)
  double2 *Sp[kPMax + 2] = {};    // sign block of A^p X0
  double first_cs[kPMax + 2][2] = {};
  double *first_sums = nullptr;  // device, 2 per power
  bool have_first = false;
  // pinned mailbox for the per-iteration results (host and device views)
  HostPost *post_host = nullptr, *post_dev = nullptr;
  unsigned long long post_seq = 0;

  // Posts v[0 .. nv), iv[0 .. ni) and *extra to the mailbox and waits for
  // them: the host spins on the sequence number (a stream synchronisation
  // costs tens of microseconds per iteration), and after 10 ms checks
  // whether the stream has stopped without posting (a device error).
  hipError_t fetch(const double *v, int nv, const int64_t *iv, int ni, const double *extra) {
    const unsigned long long seq = ++post_seq;
    hipError_t e = launch_post(v, nv, iv, ni, extra, post_dev, seq, s);
    if (e != hipSuccess) return e;
    return wait_post(seq);
  }
  hipError_t wait_post(unsigned long long seq) {
    using clock = std::chrono::steady_clock;
    auto query_at = clock::now() + std::chrono::milliseconds(10);
    for (unsigned spins = 1;; ++spins) {
      if (__atomic_load_n(&post_host->seq, __ATOMIC_ACQUIRE) == seq) return hipSuccess;
      if ((spins & 1023u) == 0 && clock::now() >= query_at) {
        const hipError_t q = hipStreamQuery(s);
        if (q != hipErrorNotReady) {
          if (__atomic_load_n(&post_host->seq, __ATOMIC_ACQUIRE) == seq) return hipSuccess;
          return q == hipSuccess ? hipErrorUnknown : q;
        }
        query_at = clock::now() + std::chrono::milliseconds(10);
      }
    }
  }

  // The probe block X0 is the same for every p, so the first iteration's
  // products A^p X0 (p = 2..pmax) come from one chain A X0, A^2 X0, ...: each
  // power's column sums and sign block are kept.  The same products in the
  // same order as in estimate(p), so the estimates are unchanged.
  hipError_t first_pass(int pmax) {
    const int t = n >= 2 ? 2 : 1;
    hipError_t e = launch_probe_init(X, n, t, s);
    if (e != hipSuccess) return e;
    const double2 *src = X;
    for (int q = 1; q <= pmax; ++q) {
      double2 *dst = (q & 1) ? W0 : W1;
      SpmvArgs a = fwd;
      a.x = src;
      a.y = dst;
      e = launch_spmm2(a, fsplit, q >= 2 ? 1 : 0, part, q >= 2 ? Sp[q] : S, h, grid, s);
      if (e != hipSuccess) return e;
      ++products;
      if (q >= 2 && (e = launch_sum_partials(part, grid, first_sums + 2 * q, s)) != hipSuccess)
        return e;
      src = dst;
    }
    e = hipMemcpyAsync(first_cs, first_sums, sizeof(first_cs), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    have_first = e == hipSuccess;
    return e;
  }

  // out = (A or A^dagger)^p in; intermediates alternate between W0 and W1,
  // the epilogue `mode` runs on the last product only.
  hipError_t power(bool adjoint, const double2 *in, double2 *out, int p, int mode) {
    const double2 *src = in;
    for (int i = 1; i <= p; ++i) {
      double2 *dst = (i == p) ? out : ((i & 1) ? W0 : W1);
      SpmvArgs a = adjoint ? adj : fwd;
      a.x = src;
      a.y = dst;
      hipError_t e = launch_spmm2(a, adjoint ? asplit : fsplit, i == p ? mode : 0, part, S, h,
                                  grid, s);
      if (e != hipSuccess) return e;
      ++products;
      src = dst;
    }
    return hipSuccess;
  }

  // Unit-column chains.  The forward products of an iteration k >= 2 start
  // from unit columns X = [e_i, e_j]; their intermediate powers A^q X are
  // kept in lad[q] (q < the chain's p), so that a later estimate whose unit
  // pair is the same, in either order, takes A^(p-1) X from there (columns
  // exchanged if need be) and computes only its last product: the same
  // products in the same order, so the estimates are unchanged.  The
  // estimates run from the largest p down, so a kept chain is at least as
  // long as a later one needs.  Null lad[1]: nothing kept.
  double2 *lad[kPMax + 1] = {};
  int lad_len = 0;                 // lad[1 .. lad_len] hold A^q X_lad
  int64_t lad_ind[2] = {-1, -1};   // X_lad = [e_lad_ind[0], e_lad_ind[1]]

  // Y = A^p [e_ind[0], e_ind[1]] (second column zero for one probe
  // column), epilogue 1.
  hipError_t forward_units(const int64_t ind[2], int p) {
    const int64_t i1 = columns() == 2 ? ind[1] : -1;
    if (!lad[1] || p < 2 || p - 1 > kPMax) {
      hipError_t e = launch_unit_cols(X, n, ind[0], i1, s);
      return e != hipSuccess ? e : power(false, X, Y, p, 1);
    }
    const bool same = ind[0] == lad_ind[0] && i1 == lad_ind[1];
    const bool swapped = i1 >= 0 && ind[0] == lad_ind[1] && i1 == lad_ind[0];
    SpmvArgs a = fwd;
    if ((same || swapped) && lad_len >= p - 1) {
      const double2 *src = lad[p - 1];
      if (swapped) {
        hipError_t e = launch_swap_pairs(W0, src, n, s);
        if (e != hipSuccess) return e;
        src = W0;
      }
      a.x = src;
      a.y = Y;
      hipError_t e = launch_spmm2(a, fsplit, 1, part, S, h, grid, s);
      if (e != hipSuccess) return e;
      ++products;
      return hipSuccess;
    }
    hipError_t e0 = launch_unit_cols(X, n, ind[0], i1, s);
    if (e0 != hipSuccess) return e0;
    lad_len = 0;
    lad_ind[0] = ind[0];
    lad_ind[1] = i1;
    const double2 *src = X;
    for (int q = 1; q <= p; ++q) {
      double2 *dst = q == p ? Y : lad[q];
      a.x = src;
      a.y = dst;
      hipError_t e = launch_spmm2(a, fsplit, q == p ? 1 : 0, part, S, h, grid, s);
      if (e != hipSuccess) return e;
      ++products;
      src = dst;
    }
    lad_len = p - 1;
    return hipSuccess;
  }

  // The decisions of one estimate (Higham and Tisseur's iteration): the
  // sequential path and the merged chains share them, so both reach the same
  // estimate from the same products.
  struct Chain {
    int p = 0, k = 1;
    double est_old = 0.0, est = 0.0;
    int64_t ind_best = -1;
    int probe_best = 0;
    int64_t ind[2] = {-1, -1};
    std::vector<int64_t> hist;
  };
  static constexpr int kItMax = 5;
  int columns() const { return n >= 2 ? 2 : 1; }
  int want(const Chain &c) const {
    return (int)std::min<int64_t>(n, (int64_t)columns() + (int64_t)c.hist.size());
  }
  static bool want_hb(const Chain &c) { return c.k >= 2 && c.ind_best >= 0; }

  // Y = A^p X of iteration c.k has column 1-norms cs: true when the estimate
  // is final, else the adjoint product follows.
  bool after_forward(Chain &c, const double cs[2]) const {
    const int t = columns();
    int jbest = 0;
    c.est = cs[0];
    if (t == 2 && cs[1] > c.est) {
      c.est = cs[1];
      jbest = 1;
    }
    if (c.est > c.est_old || c.k == 2) {
      if (c.k == 1) {
        c.ind_best = -1;
        c.probe_best = jbest;
      } else {
        c.ind_best = c.ind[jbest];
      }
    }
    if (c.k >= 2 && c.est <= c.est_old) {
      c.est = c.est_old;
      return true;
    }
    c.est_old = c.est;
    return c.k > kItMax;
  }

  // Z = (A^dagger)^p sign(Y), h_i = max_j |Z_ij|: the first `nw` indices by
  // decreasing h (ties: smaller index; values tv, indices ti) and h at
  // ind_best (hb, when want_hb) decide the next unit columns (c.ind, c.k
  // advanced); true when the estimate is final.
  bool after_adjoint(Chain &c, const double *tv, const int64_t *ti, int nw, double hb) const {
    const int t = columns();
    if (c.k >= 2 && c.ind_best >= 0 && tv[0] == hb) return true;
    auto in_hist = [&](int64_t i) {
      return std::find(c.hist.begin(), c.hist.end(), i) != c.hist.end();
    };
    if (t > 1) {
      bool all_seen = true;
      for (int j = 0; j < t && j < nw; ++j)
        if (!in_hist(ti[j])) all_seen = false;
      if (all_seen) return true;
    }
    int got = 0;
    for (int q = 0; q < nw && got < t; ++q)
      if (!in_hist(ti[q])) c.ind[got++] = ti[q];
    if (got < t) return true;
    for (int j = 0; j < t; ++j) c.hist.push_back(c.ind[j]);
    ++c.k;
    return false;
  }

  // One estimate, its products one chain at a time.
  hipError_t estimate(int p, double *est_out, int64_t *index_out, int *probe_out) {
    const int t = columns();
    const bool first_known = have_first && Sp[p] != nullptr;
    hipError_t e = first_known ? hipSuccess : launch_probe_init(X, n, t, s);
    if (e != hipSuccess) return e;
    Chain c;
    c.p = p;
    for (;;) {
      // Y = A^p X, column 1-norms and S = sign(Y) (k = 1: from first_pass)
      const bool from_first = c.k == 1 && first_known;
      const double2 *sign = from_first ? Sp[p] : S;
      double cs[2] = {0.0, 0.0};
      if (from_first) {
        cs[0] = first_cs[p][0];
        cs[1] = first_cs[p][1];
      } else {
        e = forward_units(c.ind, p);
        if (e != hipSuccess) return e;
        e = launch_sum_partials(part, grid, sums, s);
        if (e != hipSuccess) return e;
        e = fetch(sums, 2, nullptr, 0, nullptr);
        if (e != hipSuccess) return e;
        cs[0] = post_host->v[0];
        cs[1] = post_host->v[1];
      }
      if (after_forward(c, cs)) break;
      e = power(true, sign, Y, p, 2);
      if (e != hipSuccess) return e;
      const int nw = want(c);
      e = launch_topk(h, n, nw, grid, cand_v, cand_i, top_v, top_i, s);
      if (e != hipSuccess) return e;
      const bool hb_wanted = want_hb(c);
      e = fetch(top_v, nw, top_i, nw, hb_wanted ? h + c.ind_best : nullptr);
      if (e != hipSuccess) return e;
      double tv[kTopKMax];
      int64_t ti[kTopKMax];
      for (int j = 0; j < nw; ++j) {
        tv[j] = post_host->v[j];
        ti[j] = post_host->i[j];
      }
      const double hb = hb_wanted ? post_host->v[nw] : 0.0;
      if (after_adjoint(c, tv, ti, nw, hb)) break;
    }
    *est_out = c.est;
    *index_out = c.ind_best;
    *probe_out = c.probe_best;
    return hipSuccess;
  }

  // Merged chains (WideOut): wide blocks of n x 2 `width` columns (Win the
  // phase input, Wa / Wb the steps' outputs), h and column-sum partials per
  // chain.
  int width = 0;
  double2 *Win = nullptr, *Wa = nullptr, *Wb = nullptr;
  double *hc = nullptr, *partc = nullptr, *sumc = nullptr;
  double *topc_v = nullptr;
  int64_t *topc_i = nullptr;
  int wide_passes = 0;  // matrix passes of the merged chains

  // Steps 1 .. p of the chains `act` (decreasing p, slots into hc / partc /
  // Sp): Win holds their interleaved inputs; the chain with p = i finishes
  // at step i with epilogue `mode` (1: sign block into Sp[p], column-sum
  // partials; 2: h).
  hipError_t run_chains(bool adjoint, const std::vector<int> &act, const std::vector<int> &slot,
                        int mode) {
    const int m0 = (int)act.size();
    const int pmax = act[0];
    const double2 *in = Win;
    int m = m0;
    for (int i = 1; i <= pmax; ++i) {
      while (m > 0 && act[m - 1] < i) --m;  // chains still running at step i
      if (m == 0) break;
      const int fin = act[m - 1] == i ? 1 : 0;
      const int sl = slot[m - 1];
      double2 *out = (i & 1) ? Wa : Wb;
      WideOut o{};
      o.Y = out;
      o.ys = 2 * m - 2 * fin;
      o.fin = fin;
      o.mode = fin ? mode : 0;
      o.sgn = Sp[act[m - 1]];
      o.h = hc + (size_t)sl * n;
      o.part = partc + (size_t)sl * 2 * grid;
      SpmvArgs a = adjoint ? adj : fwd;
      a.x = in;
      a.y = nullptr;
      hipError_t e = launch_spmm_wide(a, adjoint ? asplit : fsplit, 2 * m, o, grid, s);
      if (e != hipSuccess) return e;
      products += m;
      ++wide_passes;
      in = out;
    }
    return hipSuccess;
  }

  // The estimates of ps (decreasing p) together, after first_pass; the
  // results are those of estimate(p) for each p, bit for bit.
  hipError_t estimate_merged(const std::vector<int> &ps, double *est_out, int64_t *index_out,
                             int *probe_out) {
    const int g = (int)ps.size();
    const int t = columns();
    if (g < 1 || g > width || t != 2) return hipErrorInvalidValue;
    std::vector<Chain> ch(g);
    std::vector<bool> done(g, false);
    for (int j = 0; j < g; ++j) {
      ch[j].p = ps[j];
      done[j] = after_forward(ch[j], first_cs[ps[j]]);
    }
    hipError_t e = hipSuccess;
    for (bool adjoint = true;; adjoint = !adjoint) {
      std::vector<int> act, slot;
      for (int j = 0; j < g; ++j)
        if (!done[j]) {
          act.push_back(ps[j]);
          slot.push_back(j);
        }
      if (act.empty()) break;
      const int m = (int)act.size();
      if (adjoint) {
        PairSources src{};
        src.chains = m;
        for (int q = 0; q < m; ++q) src.src[q] = Sp[act[q]];
        if ((e = launch_pack_pairs(Win, n, src, s)) != hipSuccess) return e;
        if ((e = run_chains(true, act, slot, 2)) != hipSuccess) return e;
        PostList pl{};
        pl.chains = m;
        for (int q = 0; q < m; ++q) {
          const Chain &c = ch[slot[q]];
          const int nw = want(c);
          double *tv = topc_v + (size_t)q * kTopKMax;
          int64_t *ti = topc_i + (size_t)q * kTopKMax;
          const double *hq = hc + (size_t)slot[q] * n;
          if ((e = launch_topk(hq, n, nw, grid, cand_v, cand_i, tv, ti, s)) != hipSuccess) return e;
          pl.v[q] = tv;
          pl.i[q] = ti;
          pl.nv[q] = nw;
          pl.ni[q] = nw;
          pl.extra[q] = want_hb(c) ? hq + c.ind_best : nullptr;
        }
        const unsigned long long seq = ++post_seq;
        if ((e = launch_post_list(pl, post_dev, seq, s)) != hipSuccess) return e;
        if ((e = wait_post(seq)) != hipSuccess) return e;
        for (int q = 0; q < m; ++q) {
          Chain &c = ch[slot[q]];
          const int nw = pl.nv[q];
          const double *pv = post_host->v + q * (kTopKMax + 1);
          const int64_t *pi = post_host->i + q * kTopKMax;
          double tv[kTopKMax];
          int64_t ti[kTopKMax];
          for (int j = 0; j < nw; ++j) {
            tv[j] = pv[j];
            ti[j] = pi[j];
          }
          const double hb = pl.extra[q] ? pv[nw] : 0.0;
          done[slot[q]] = after_adjoint(c, tv, ti, nw, hb);
        }
      } else {
        PairUnits pu{};
        pu.chains = m;
        for (int q = 0; q < m; ++q) {
          pu.ind[q][0] = ch[slot[q]].ind[0];
          pu.ind[q][1] = ch[slot[q]].ind[1];
        }
        if ((e = launch_unit_pairs(Win, n, pu, s)) != hipSuccess) return e;
        if ((e = run_chains(false, act, slot, 1)) != hipSuccess) return e;
        for (int q = 0; q < m; ++q)
          if ((e = launch_sum_partials(partc + (size_t)slot[q] * 2 * grid, grid, sumc + 2 * q,
                                       s)) != hipSuccess)
            return e;
        if ((e = fetch(sumc, 2 * m, nullptr, 0, nullptr)) != hipSuccess) return e;
        for (int q = 0; q < m; ++q) {
          const double cs[2] = {post_host->v[2 * q], post_host->v[2 * q + 1]};
          done[slot[q]] = after_forward(ch[slot[q]], cs);
        }
      }
    }
    for (int j = 0; j < g; ++j) {
      est_out[j] = ch[j].est;
      index_out[j] = ch[j].ind_best;
      probe_out[j] = ch[j].probe_best;
    }
    return hipSuccess;
  }
};

// Wave-jagged execution layout (see kWaveRows) of one CSR.
// Complex values (val) or phase-split values (coef, diag; split = true),
// with block-shared leading positions (sh) when split.
struct WaveLayout {
  int32_t *col = nullptr;
  double2 *val = nullptr;
  double *coef = nullptr;
  double2 *diag = nullptr;
  bool split = false;
  int32_t *len = nullptr;
  unsigned char *perm = nullptr;
  int32_t *glob = nullptr;
  int32_t *shn = nullptr;
  int64_t *start = nullptr, *shs = nullptr;
  SharedEntry *sh = nullptr;
  int32_t stride = 0;   // shared entries of block k at sh + k stride
  int64_t nwb = 0;
  int64_t entries = 0;  // per-row entries stored (without the shared positions)
  int64_t shared = 0;   // shared entries read per product (padded counts)
  int64_t distinct = 0; // per-row entries in the copies the blocks read (after dedup)
  void release_values() {
    dfree(col);
    dfree(val);
    dfree(coef);
    dfree(diag);
    dfree(sh);
  }
  void release() {
    release_values();
    dfree(len);
    dfree(perm);
    dfree(glob);
    dfree(shn);
    dfree(start);
    dfree(shs);
  }
};

// Point every block whose stored rows equal an earlier block's (same
// lengths after the shared positions, same words, same split position) at
// that block's copy, so the blocks read one copy (cached) instead of their
// own.  Candidates come from a hash; each is compared in full on the device.
hipError_t dedup_blocks(WaveLayout &W, int64_t n, const std::vector<int64_t> &hcnt,
                        const std::vector<int32_t> &hshn, const std::vector<int64_t> &hstart,
                        hipStream_t s) {
  const size_t nwb = (size_t)W.nwb;
  if (nwb < 2) return hipSuccess;
  unsigned long long *hash = nullptr;
  int64_t *canon = nullptr;
  int *same = nullptr;
  hipError_t e;
  std::vector<unsigned long long> hh(nwb);
  std::vector<int32_t> hglob(nwb);
  std::vector<int64_t> hcanon(nwb);
  std::vector<int> hsame(nwb);
  do {
    if ((e = dalloc(&hash, nwb)) != hipSuccess) break;
    if ((e = dalloc(&canon, nwb)) != hipSuccess) break;
    if ((e = dalloc(&same, nwb)) != hipSuccess) break;
    if ((e = launch_wjag_hash(W.col, W.coef, W.val, W.len, W.shn, W.start, n, hash, s)) !=
        hipSuccess)
      break;
    if ((e = hipMemcpyAsync(hh.data(), hash, nwb * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
      break;
    if ((e = hipMemcpyAsync(hglob.data(), W.glob, nwb * sizeof(int32_t), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    // key: hash, stored entries, split position within the stored rows; the
    // first block of each key (the smallest index) is its candidate copy
    struct Key {
      unsigned long long h;
      int64_t cnt;
      int32_t g;
      bool operator==(const Key &o) const { return h == o.h && cnt == o.cnt && g == o.g; }
    };
    struct KeyHash {
      size_t operator()(const Key &k) const {
        return (size_t)(k.h ^ ((unsigned long long)k.cnt * 0x9E3779B97F4A7C15ull) ^
                        ((unsigned long long)(uint32_t)k.g << 17));
      }
    };
    std::unordered_map<Key, int64_t, KeyHash> first;
    first.reserve(nwb);
    int64_t dup = 0;
    for (size_t k = 0; k < nwb; ++k) {
      const int32_t g = hglob[k] < 0 ? -1 : (hglob[k] & kGlobMask) - hshn[k];
      auto it = first.emplace(Key{hh[k], hcnt[k], g}, (int64_t)k).first;
      hcanon[k] = it->second;
      dup += it->second != (int64_t)k;
    }
    if (dup == 0) break;
    if ((e = hipMemcpyAsync(canon, hcanon.data(), nwb * sizeof(int64_t), hipMemcpyHostToDevice,
                            s)) != hipSuccess)
      break;
    if ((e = launch_wjag_same(W.col, W.coef, W.val, W.len, W.shn, W.start, n, canon, same, s)) !=
        hipSuccess)
      break;
    if ((e = hipMemcpyAsync(hsame.data(), same, nwb * sizeof(int), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    std::vector<int64_t> start(hstart);
    for (size_t k = 0; k < nwb; ++k)
      if (hsame[k]) {
        start[k] = hstart[(size_t)hcanon[k]];
        W.distinct -= hcnt[k];
      }
    if ((e = hipMemcpyAsync(W.start, start.data(), nwb * sizeof(int64_t), hipMemcpyHostToDevice,
                            s)) != hipSuccess)
      break;
    e = hipStreamSynchronize(s);
  } while (false);
  dfree(hash);
  dfree(canon);
  dfree(same);
  return e;
}

// Phase-split values with block-shared positions unless an off-diagonal
// entry is neither real nor imaginary (then complex values); blocks with
// equal stored rows read one copy.  QSW_SPLIT=0, QSW_SHARED=0 and
// QSW_DEDUP=0 turn each off.
hipError_t build_wave_layout(const int64_t *rp, const int32_t *col, const double2 *val, int64_t n,
                             int64_t nnz, int32_t N, hipStream_t s, WaveLayout &W) {
  (void)nnz;
  hipError_t e;
  W.nwb = (n + kWaveRows - 1) / kWaveRows;
  const size_t nwb = (size_t)W.nwb;
  if ((e = dalloc(&W.len, (size_t)n)) != hipSuccess) return e;
  if ((e = dalloc(&W.perm, (size_t)n)) != hipSuccess) return e;
  if ((e = dalloc(&W.glob, nwb)) != hipSuccess) return e;
  if ((e = dalloc(&W.shn, nwb)) != hipSuccess) return e;
  if ((e = dalloc(&W.start, nwb + 1)) != hipSuccess) return e;
  if ((e = dalloc(&W.shs, nwb + 1)) != hipSuccess) return e;
  int64_t *cnt = nullptr;
  int *bad = nullptr;
  if ((e = dalloc(&cnt, nwb)) != hipSuccess) return e;
  if ((e = dalloc(&bad, 1)) != hipSuccess) {
    dfree(cnt);
    return e;
  }
  std::vector<int32_t> hshn(nwb);
  std::vector<int64_t> hcnt(nwb), hstart(nwb + 1), hshs(nwb + 1);
  const bool try_split = n <= kSplitMaxN && env_int("QSW_SPLIT", 1) != 0;
  for (int attempt = try_split ? 1 : 0; attempt >= 0; --attempt) {
    const bool split = attempt == 1;
    const bool shared = split && env_int("QSW_SHARED", 1) != 0;
    int hbad = 0;
    do {
      if ((e = launch_wjag_plan(rp, col, val, n, N, shared, W.glob, W.shn, cnt, s)) != hipSuccess)
        break;
      if ((e = hipMemcpyAsync(hshn.data(), W.shn, nwb * sizeof(int32_t), hipMemcpyDeviceToHost,
                              s)) != hipSuccess)
        break;
      if ((e = hipMemcpyAsync(hcnt.data(), cnt, nwb * sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
        break;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
      // shared entries at a fixed stride per block (the largest padded
      // count): a block's address is known before its header is read
      hstart[0] = 0;
      int64_t padded = 0;
      int32_t stride = 0;
      for (size_t k = 0; k < nwb; ++k) {
        hstart[k + 1] = hstart[k] + hcnt[k];
        const int32_t pc = (hshn[k] + kSharedPad - 1) / kSharedPad * kSharedPad;
        padded += pc;
        stride = std::max(stride, pc);
      }
      for (size_t k = 0; k <= nwb; ++k) hshs[k] = (int64_t)k * stride;
      W.stride = stride;
      W.entries = W.distinct = hstart[nwb];
      W.shared = padded;
      if ((e = hipMemcpyAsync(W.start, hstart.data(), (nwb + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, s)) != hipSuccess)
        break;
      if ((e = hipMemcpyAsync(W.shs, hshs.data(), (nwb + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, s)) != hipSuccess)
        break;
      // kWavePad zero entries (offset 0, value 0) after the last one: the
      // product loops read up to 63 entries past a block's end
      const size_t ent = (size_t)W.entries + kWavePad;
      if ((e = dalloc(&W.col, ent)) != hipSuccess) break;
      if ((e = launch_zero(W.col + W.entries, kWavePad * sizeof(int32_t), s)) != hipSuccess) break;
      if (split) {
        if ((e = dalloc(&W.coef, ent)) != hipSuccess) break;
        if ((e = launch_zero(W.coef + W.entries, kWavePad * sizeof(double), s)) != hipSuccess) break;
        if ((e = dalloc(&W.diag, (size_t)n)) != hipSuccess) break;
      } else {
        if ((e = dalloc(&W.val, ent)) != hipSuccess) break;
        if ((e = launch_zero(W.val + W.entries, kWavePad * sizeof(double2), s)) != hipSuccess) break;
      }
      if ((e = dalloc(&W.sh, std::max<size_t>(1, (size_t)nwb * (size_t)W.stride))) != hipSuccess)
        break;
      if ((e = launch_zero(bad, sizeof(int), s)) != hipSuccess) break;
      if ((e = launch_wjag_fill(rp, col, val, n, N, split, W.shn, W.start, W.shs, W.col, W.val,
                                W.coef, W.diag, W.len, W.perm, W.sh, bad, s)) != hipSuccess)
        break;
      if ((e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
        break;
      e = hipStreamSynchronize(s);
    } while (false);
    if (e != hipSuccess) break;
    if (!split || !hbad) {
      W.split = split;
      if (env_int("QSW_DEDUP", 1) != 0) e = dedup_blocks(W, n, hcnt, hshn, hstart, s);
      break;
    }
    W.release_values();  // an entry neither real nor imaginary: complex values
  }
  dfree(cnt);
  dfree(bad);
  return e;
}

void set_wave(SpmvArgs &a, const WaveLayout &W) {
  a.nwb = W.nwb;
  a.wcol = W.col;
  a.wval = W.val;
  a.wcoef = W.coef;
  a.wdiag = W.diag;
  a.wlen = W.len;
  a.wperm = W.perm;
  a.wglob = W.glob;
  a.wstart = W.start;
  a.wshn = W.shared > 0 ? W.shn : nullptr;
  a.wshs = W.shs;
  a.wsh = W.sh;
  a.wsh_stride = W.stride;
}

void set_wave(SpmvArgs &a, const qsw_superop_s *h) {
  a.nwb = h->nwb;
  a.N = h->N;
  a.wcol = h->wcol;
  a.wval = h->wval;
  a.wval32 = h->wval32;
  a.wcoef = h->wcoef;
  a.wcoef32 = h->wcoef32;
  a.wdiag = h->wdiag;
  a.wdiag32 = h->wdiag32;
  a.wlen = h->wlen;
  a.wperm = h->wperm;
  a.wglob = h->wglob;
  a.wstart = h->wstart;
  a.wshn = h->wshared > 0 ? h->wshn : nullptr;
  a.wshs = h->wshs;
  a.wsh = h->wsh;
  a.wsh_stride = h->wsh_stride;
}

// The XCD-banded engine needs N/64 blocks per rho-row in 8 bands and at most
// 32 KB of staged rows: N = 512, 1024 or 2048.
bool banded_ok(int32_t N) {
  return kBlockThreads == 256 && (N == 512 || N == 1024 || N == 2048);
}

// Its grid: a multiple of the 8 XCDs.
int banded_grid(int grid) { return std::max(8, grid / 8 * 8); }

// Workgroups of a wave-jagged launch: one wavefront per block up to twice
// the resident capacity, then blocks per wavefront grow.
int wave_grid(int64_t nwb, int resident) {
  const int64_t wgs = (nwb + kBlockThreads / 64 - 1) / (kBlockThreads / 64);
  // about two rounds of resident workgroups, each taking its quads
  // grid-stride, with the quads split evenly: q = ceil(quads / cap) quads per
  // workgroup and ceil(quads / q) workgroups.  On the 1024-vertex operator
  // (4096 quads) a pass took 104.7 ms at 2048 workgroups (two quads each),
  // 106.4 at 2560 (an uneven split), 111.5 at 3584 and 109.8 at 4096 (one
  // quad each); single-precision products 58.1, 59.2, 68.2 and 69.6 ms.
  // Later kernels: 91.5 ms at 2048, 94.5 at 1024 (four quads each), 107.6
  // at 1366 (three) and 101.6 at 4096, the same results bit for bit.
  int64_t cap = 2 * (int64_t)std::max(resident, 1);
  cap = std::max<int64_t>(1, env_int("QSW_GRID", (int)cap));
  const int64_t q = (wgs + cap - 1) / cap;
  return (int)std::max<int64_t>(1, (wgs + q - 1) / std::max<int64_t>(q, 1));
}

// H (Hermitian, complex, may hold a diagonal) into the off-diagonal CSR and
// diagonal of HostOps; checks pattern symmetry and H_ji = conj(H_ij).
qsw_status_t parse_hermitian(int32_t N, const int64_t *rp, const int32_t *ci, const double *v,
                             HostOps &op) {
  const int64_t E = rp[N];
  if (E > 0 && (!ci || !v)) return QSW_ERR_ARG;
  qsw_status_t st = check_csr(N, rp, ci, true);
  if (st != QSW_OK) return st;
  op.hp.assign(N + 1, 0);
  op.hdiag.assign(N, 0.0);
  for (int32_t i = 0; i < N; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const double re = v[2 * e], im = v[2 * e + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return QSW_ERR_GRAPH;
      if (ci[e] == i) {
        if (std::fabs(im) > 1e-14 * (1.0 + std::fabs(re))) return QSW_ERR_GRAPH;  // not Hermitian
        op.hdiag[i] = re;
      } else {
        op.hc.push_back(ci[e]);
        op.hv.push_back(re);
        op.hv.push_back(im);
      }
    }
    op.hp[i + 1] = (int64_t)op.hc.size();
  }
  for (int32_t i = 0; i < N; ++i)
    for (int64_t e = op.hp[i]; e < op.hp[i + 1]; ++e) {
      const int32_t j = op.hc[e];
      const auto b = op.hc.begin() + op.hp[j], en = op.hc.begin() + op.hp[j + 1];
      const auto it = std::lower_bound(b, en, i);
      if (it == en || *it != i) return QSW_ERR_GRAPH;
      const int64_t f = it - op.hc.begin();
      const double tolh = 1e-14 * (1.0 + std::fabs(op.hv[2 * e]) + std::fabs(op.hv[2 * e + 1]));
      if (std::fabs(op.hv[2 * f] - op.hv[2 * e]) > tolh ||
          std::fabs(op.hv[2 * f + 1] + op.hv[2 * e + 1]) > tolh)
        return QSW_ERR_GRAPH;
    }
  return QSW_OK;
}

// A real coefficient matrix M (each entry one L_k = M_ij |i><j|) into rates
// |M_ij|^2: off-diagonal CSR plus diagonal.
qsw_status_t parse_rates(int32_t N, const int64_t *rp, const int32_t *ci, const double *v,
                         std::vector<int64_t> &op_rp, std::vector<int32_t> &op_rc,
                         std::vector<double> &op_rv, std::vector<double> &op_rdiag) {
  const int64_t E = rp[N];
  if (E > 0 && (!ci || !v)) return QSW_ERR_ARG;
  qsw_status_t st = check_csr(N, rp, ci, true);
  if (st != QSW_OK) return st;
  op_rp.assign(N + 1, 0);
  op_rdiag.assign(N, 0.0);
  for (int32_t i = 0; i < N; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const double x = v[e];
      if (!std::isfinite(x)) return QSW_ERR_GRAPH;
      if (ci[e] == i) {
        op_rdiag[i] = x * x;
      } else if (x != 0.0) {
        op_rc.push_back(ci[e]);
        op_rv.push_back(x * x);
      }
    }
    op_rp[i + 1] = (int64_t)op_rc.size();
  }
  return QSW_OK;
}

}  // namespace

// What a handle is built from, kept so that qsw_superop_set_omega can
// rebuild it: assembles L (or its adjoint) for a given omega into fresh
// device CSR arrays.
struct qsw::Assembler {
  virtual ~Assembler() {}
  virtual int32_t order() const = 0;
  virtual int64_t max_row(double omega) const = 0;
  virtual qsw_status_t assemble(bool adjoint, double omega, hipStream_t s, int64_t **rp,
                                int32_t **col, double2 **val, int64_t *nnz) const = 0;
  // Walks whose L^dagger differs from L only as the adjoint products through
  // L's layout assume (a real H; population transfers only in the rows
  // (a, a)): frp, the row pointer of L's rates, and trp / tcol / tval, the
  // transposed rates with the values L^dagger's assembly writes (row a:
  // omega R_ja for rho_jj, ascending j).  False: L^dagger is assembled.
  virtual bool adjoint_transfers(double omega, std::vector<int64_t> &frp,
                                 std::vector<int64_t> &trp, std::vector<int32_t> &tcol,
                                 std::vector<double> &tval) const {
    (void)omega, (void)frp, (void)trp, (void)tcol, (void)tval;
    return false;
  }
};

namespace {

// Walks of the local-interaction family (eq. qsw, plus rates outside omega
// for absorption and emission, eq. qsw_ss): assembled on the device.
struct LocalAssembler : Assembler {
  HostOps op;
  int32_t order() const override { return op.N; }
  int64_t max_row(double omega) const override {
    return max_row_bound(op, effective_rates(op, omega));
  }
  qsw_status_t assemble(bool adjoint, double omega, hipStream_t s, int64_t **rp, int32_t **col,
                        double2 **val, int64_t *nnz) const override {
    return ::assemble(op, effective_rates(op, omega), adjoint, omega, s, rp, col, val, nnz);
  }
  bool adjoint_transfers(double omega, std::vector<int64_t> &frp, std::vector<int64_t> &trp,
                         std::vector<int32_t> &tcol, std::vector<double> &tval) const override {
    for (size_t i = 1; i < op.hv.size(); i += 2)
      if (op.hv[i] != 0.0) return false;  // a complex H: its entries are not all imaginary in L
    const Rates R = effective_rates(op, omega);
    std::vector<double> rtv;
    // as assemble(adjoint = true) transposes them, and each value as its
    // kernel scales it
    transpose_csr(op.N, R.rp, R.rc, R.rv, 1, trp, tcol, rtv);
    tval.resize(rtv.size());
    for (size_t e = 0; e < rtv.size(); ++e) tval[e] = R.scale * rtv[e];
    frp = R.rp;
    return true;
  }
};

// Complex host CSR (rows sorted, no duplicates) of an N x N operator.
struct HostCsr {
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<std::complex<double>> val;
};

// A complex host CSR (interleaved values); `hermitian` also checks
// H_ji = conj(H_ij) for every stored entry.
qsw_status_t parse_complex(int32_t N, const int64_t *rp, const int32_t *ci, const double *v,
                           bool hermitian, HostCsr &A) {
  if (!rp) return QSW_ERR_ARG;
  const int64_t E = rp[N];
  if (E > 0 && (!ci || !v)) return QSW_ERR_ARG;
  qsw_status_t st = check_csr(N, rp, ci, true);
  if (st != QSW_OK) return st;
  A.rp.assign(rp, rp + N + 1);
  A.col.assign(ci, ci + E);
  A.val.resize(E);
  for (int64_t e = 0; e < E; ++e) {
    if (!std::isfinite(v[2 * e]) || !std::isfinite(v[2 * e + 1])) return QSW_ERR_GRAPH;
    A.val[e] = {v[2 * e], v[2 * e + 1]};
  }
  if (hermitian)
    for (int32_t i = 0; i < N; ++i)
      for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
        const int32_t j = A.col[e];
        const auto b = A.col.begin() + A.rp[j], en = A.col.begin() + A.rp[j + 1];
        const auto it = std::lower_bound(b, en, i);
        if (it == en || *it != i) return QSW_ERR_GRAPH;
        const std::complex<double> x = A.val[e], y = A.val[it - A.col.begin()];
        if (std::abs(y - std::conj(x)) > 1e-14 * (1.0 + std::abs(x))) return QSW_ERR_GRAPH;
      }
  return QSW_OK;
}

HostCsr conj_transpose(int32_t N, const HostCsr &A) {
  HostCsr T;
  T.rp.assign(N + 1, 0);
  for (int32_t c : A.col) T.rp[c + 1]++;
  for (int32_t i = 0; i < N; ++i) T.rp[i + 1] += T.rp[i];
  T.col.resize(A.col.size());
  T.val.resize(A.col.size());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int32_t i = 0; i < N; ++i)
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int64_t o = pos[A.col[e]]++;
      T.col[o] = i;
      T.val[o] = std::conj(A.val[e]);
    }
  return T;
}

HostCsr product(int32_t N, const HostCsr &A, const HostCsr &B) {  // A B
  HostCsr C;
  C.rp.assign(N + 1, 0);
  std::vector<std::complex<double>> acc(N);
  std::vector<char> used(N, 0);
  std::vector<int32_t> cols;
  for (int32_t i = 0; i < N; ++i) {
    cols.clear();
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int32_t k = A.col[e];
      for (int64_t f = B.rp[k]; f < B.rp[k + 1]; ++f) {
        const int32_t j = B.col[f];
        if (!used[j]) {
          used[j] = 1;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += A.val[e] * B.val[f];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      C.col.push_back(j);
      C.val.push_back(acc[j]);
      used[j] = 0;
    }
    C.rp[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

// Walks given by explicit operators (the global-interaction family):
//   L = -i(1-omega)[H, .] + omega ( i[H_rot, .] + sum_k D[L_k] )
// (eq. qsw with one or more general L_k, eq. nm_gqsw with H_rot), assembled
// on the host as Kronecker terms in the row-major vec(rho)_(aN+b) = rho_ab:
// A rho B -> A kron B^T.  Its explicit entries are those of the terms'
// patterns (zeros kept), so the pattern does not depend on omega.
struct GeneralAssembler : Assembler {
  int32_t N = 0;
  HostCsr H, Hrot;
  std::vector<HostCsr> Ls, LdLs;  // L_k and L_k^dagger L_k
  int32_t order() const override { return N; }

  // One row r = a N + b of L (sigma = +1) or of L^dagger: (col, val) pairs,
  // merged.  For the adjoint every operator is replaced by its adjoint
  // (H, H_rot: -i -> +i; L_k rho L_k^dag -> L_k^dag rho L_k).
  void row(int64_t a, int64_t b, double omega, bool adjoint, std::vector<int64_t> &c,
           std::vector<std::complex<double>> &v, const std::vector<HostCsr> &Lt) const {
    const std::complex<double> I(0.0, 1.0);
    const double sg = adjoint ? -1.0 : 1.0;
    auto commutator = [&](const HostCsr &M, std::complex<double> f) {
      // f (M rho - rho M): M kron I and I kron M^T
      for (int64_t e = M.rp[a]; e < M.rp[a + 1]; ++e) {
        c.push_back((int64_t)M.col[e] * N + b);
        v.push_back(f * M.val[e]);
      }
      // (rho M)_ab = sum_d rho_ad M_db: column a N + d over M's column b, i.e.
      // the row b of M^T; M is Hermitian here so M_db = conj(M_bd)
      for (int64_t e = M.rp[b]; e < M.rp[b + 1]; ++e) {
        c.push_back(a * N + M.col[e]);
        v.push_back(-f * std::conj(M.val[e]));
      }
    };
    commutator(H, sg * -I * (1.0 - omega));
    if (!Hrot.rp.empty()) commutator(Hrot, sg * I * omega);
    for (size_t k = 0; k < Ls.size(); ++k) {
      // L rho L^dag -> (L kron conj(L)); for the adjoint L^dag rho L -> (L^dag kron L^T)
      const HostCsr &A = adjoint ? Lt[k] : Ls[k];
      for (int64_t e = A.rp[a]; e < A.rp[a + 1]; ++e)
        for (int64_t f = A.rp[b]; f < A.rp[b + 1]; ++f) {
          c.push_back((int64_t)A.col[e] * N + A.col[f]);
          v.push_back(omega * A.val[e] * std::conj(A.val[f]));
        }
      // -1/2 {L^dag L, rho}; L^dag L is Hermitian, the same for the adjoint
      const HostCsr &M = LdLs[k];
      for (int64_t e = M.rp[a]; e < M.rp[a + 1]; ++e) {
        c.push_back((int64_t)M.col[e] * N + b);
        v.push_back(-0.5 * omega * M.val[e]);
      }
      for (int64_t e = M.rp[b]; e < M.rp[b + 1]; ++e) {
        c.push_back(a * N + M.col[e]);
        v.push_back(-0.5 * omega * std::conj(M.val[e]));
      }
    }
  }

  int64_t max_row(double) const override { return 0; }  // exact lengths are known

  qsw_status_t assemble(bool adjoint, double omega, hipStream_t s, int64_t **rp_out,
                        int32_t **col_out, double2 **val_out, int64_t *nnz_out) const override {
    const int64_t n = (int64_t)N * N;
    std::vector<HostCsr> Lt;
    if (adjoint)
      for (const HostCsr &L : Ls) Lt.push_back(conj_transpose(N, L));
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int64_t> c;
    std::vector<std::complex<double>> v;
    std::vector<std::pair<int64_t, std::complex<double>>> ent;
    for (int64_t a = 0; a < N; ++a)
      for (int64_t b = 0; b < N; ++b) {
        c.clear();
        v.clear();
        row(a, b, omega, adjoint, c, v, Lt);
        ent.resize(c.size());
        for (size_t i = 0; i < c.size(); ++i) ent[i] = {c[i], v[i]};
        std::sort(ent.begin(), ent.end(),
                  [](const auto &x, const auto &y) { return x.first < y.first; });
        for (size_t i = 0; i < ent.size();) {
          std::complex<double> acc = 0.0;
          size_t j = i;
          // summed in a fixed order: the sort is by column, ties in term order
          for (; j < ent.size() && ent[j].first == ent[i].first; ++j) acc += ent[j].second;
          col.push_back((int32_t)ent[i].first);
          val.push_back(acc.real());
          val.push_back(acc.imag());
          i = j;
        }
        rp[a * N + b + 1] = (int64_t)col.size();
      }
    const int64_t nnz = (int64_t)col.size();
    int64_t *drp = nullptr;
    int32_t *dcol = nullptr;
    double2 *dval = nullptr;
    hipError_t e = hipSuccess;
    do {
      if ((e = upload(&drp, rp, s)) != hipSuccess) break;
      if ((e = upload(&dcol, col, s)) != hipSuccess) break;
      if ((e = dalloc(&dval, (size_t)nnz)) != hipSuccess) break;
      if (nnz && (e = hipMemcpyAsync(dval, val.data(), val.size() * sizeof(double),
                                     hipMemcpyHostToDevice, s)) != hipSuccess)
        break;
      e = hipStreamSynchronize(s);  // the host vectors must outlive the copies
    } while (false);
    if (e != hipSuccess) {
      dfree(drp);
      dfree(dcol);
      dfree(dval);
      return status_of(e);
    }
    *rp_out = drp;
    *col_out = dcol;
    *val_out = dval;
    *nnz_out = nnz;
    return QSW_OK;
  }
};

qsw_status_t build_common(std::shared_ptr<Assembler> src, double omega, hipStream_t s,
                          qsw_superop_t *out) {
  auto t_start = std::chrono::steady_clock::now();
  const int32_t N = src->order();
  const int64_t n = (int64_t)N * N;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  qsw_superop_s *h = new (std::nothrow) qsw_superop_s();
  if (!h) return QSW_ERR_OOM;
  h->device = dev;
  h->N = N;
  h->n = n;
  h->omega = omega;
  h->src = src;
  auto fail = [&](qsw_status_t st) {
    qsw_superop_destroy(h);
    return st;
  };
  qsw_status_t st = src->assemble(false, omega, s, &h->row_ptr, &h->col, &h->val, &h->nnz);
  if (st != QSW_OK) return fail(st);
  // product-kernel layout of L (stream engine unless QSW_ENGINE selects the
  // vector engine with that many lanes per row)
  int64_t maxrow = src->max_row(omega);
  if (maxrow <= 0) {  // read the longest row from the row pointer
    std::vector<int64_t> rph((size_t)n + 1);
    HIP_TRY(hipMemcpy(rph.data(), h->row_ptr, rph.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < n; ++r) maxrow = std::max(maxrow, rph[r + 1] - rph[r]);
  }
  const int resident1 = resident_workgroups(0);
  {
    Layout L;
    hipError_t le =
        make_layout(h->row_ptr, n, h->nnz, maxrow, kCap, resident_workgroups(2), s, L);
    if (le != hipSuccess) {
      dfree(L.blk);
      return fail(status_of(le));
    }
    h->blk = L.blk;
    h->nblk = L.nblk;
    h->blocks_per_wg = L.bpw;
    // wave-jagged copy for the product kernels
    WaveLayout W;
    hipError_t we = build_wave_layout(h->row_ptr, h->col, h->val, h->n, h->nnz, N, s, W);
    h->wcol = W.col;
    h->wval = W.val;
    h->wcoef = W.coef;
    h->wdiag = W.diag;
    h->split = W.split;
    h->wlen = W.len;
    h->wperm = W.perm;
    h->wglob = W.glob;
    h->wshn = W.shn;
    h->wstart = W.start;
    h->wshs = W.shs;
    h->wsh = W.sh;
    h->wsh_stride = W.stride;
    h->wentries = W.entries;
    h->wshared = W.shared;
    h->wdistinct = W.distinct;
    if (we != hipSuccess) return fail(status_of(we));
    h->nwb = W.nwb;
    const int eng = env_int("QSW_ENGINE", 0);
    // stage the rho-row in LDS when it is small enough to leave the
    // occupancy alone (QSW_STAGE=0 turns it off)
    const bool stage = (size_t)N * sizeof(double2) <= kStageMaxBytes && env_int("QSW_STAGE", 1) != 0;
    h->engine = stage ? 100 : 0;
    h->grid = wave_grid(h->nwb, resident1);
    // the XCD-banded traversal measured no faster than plain staging on the
    // 1024-vertex workloads, so it is taken only on request (QSW_BANDS=1) or
    // when the autotuner finds it faster
    if (stage && banded_ok(N) && env_int("QSW_BANDS", 0) != 0) {
      h->engine = 200;
      h->grid = banded_grid(h->grid);
    }
    // long rows (at least kWideRowEntries stored entries per row on average)
    // take wide groups at four waves per SIMD (QSW_WIDE=1 always, 0 never)
    const int wide = env_int("QSW_WIDE", -1);
    if (stage && h->engine == 100 &&
        (wide > 0 || (wide < 0 && h->n > 0 && h->wentries >= kWideRowEntries * h->n)))
      h->engine = 300;
    if (eng == 3) {
      h->engine = 3;
      h->grid = L.grid;
    } else if (eng == 4 || eng == 8 || eng == 16 || eng == 32 || eng == 64) {
      choose_vector_launch(h, eng);
    }
  }
  // L^dagger for ||L||_1 and the estimator: through the phase-split layout
  // of L where the walk allows it (no CSR or layout of its own; the same
  // values bit for bit, QSW_ADJ_LAYOUT=1 assembles it anyway), else
  // assembled and laid out
  std::vector<int64_t> hfrp, htrp;
  std::vector<int32_t> htcol;
  std::vector<double> htval;
  const bool adj_fwd = h->split && env_int("QSW_ADJ_LAYOUT", 0) == 0 &&
                       src->adjoint_transfers(omega, hfrp, htrp, htcol, htval);
  int64_t *arp = nullptr;
  int32_t *acol = nullptr;
  double2 *aval = nullptr;
  int64_t annz = 0;
  if (!adj_fwd) {
    st = src->assemble(true, omega, s, &arp, &acol, &aval, &annz);
    if (st != QSW_OK) return fail(st);
  }
  int64_t *dfrp = nullptr, *dtrp = nullptr;
  int32_t *dtcol = nullptr;
  double *dtval = nullptr;
  unsigned long long *nbits = nullptr;
  Estimator E{};
  WaveLayout WA;
  hipError_t e = hipSuccess;
  double norm1 = 0.0;
  do {
    if ((e = dalloc(&nbits, 1)) != hipSuccess) break;
    if ((e = launch_zero(nbits, sizeof(unsigned long long), s)) != hipSuccess) break;
    if (adj_fwd) {
      const size_t nt = std::max<size_t>(htcol.size(), 1);
      if ((e = dalloc(&dfrp, hfrp.size())) != hipSuccess) break;
      if ((e = dalloc(&dtrp, htrp.size())) != hipSuccess) break;
      if ((e = dalloc(&dtcol, nt)) != hipSuccess) break;
      if ((e = dalloc(&dtval, nt)) != hipSuccess) break;
      // the host vectors outlive the copies (the stream is synchronised below)
      if ((e = hipMemcpyAsync(dfrp, hfrp.data(), hfrp.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(dtrp, htrp.data(), htrp.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s)) != hipSuccess) break;
      if (!htcol.empty() &&
          ((e = hipMemcpyAsync(dtcol, htcol.data(), htcol.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s)) != hipSuccess ||
           (e = hipMemcpyAsync(dtval, htval.data(), htval.size() * sizeof(double),
                               hipMemcpyHostToDevice, s)) != hipSuccess)) break;
      if ((e = launch_adj_row_abs_max(n, N, h->row_ptr, h->val, dfrp, dtrp, dtval, nbits, s)) !=
          hipSuccess) break;
    } else if ((e = launch_row_abs_max(n, arp, aval, nbits, s)) != hipSuccess) {
      break;
    }
    unsigned long long bits = 0;
    if ((e = hipMemcpyAsync(&bits, nbits, sizeof(bits), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    std::memcpy(&norm1, &bits, sizeof(double));
    h->info.norm1 = norm1;
    h->info.d[0] = h->info.d[1] = norm1;
    for (int p = 0; p < 10; ++p) {
      h->info.d_index[p] = -1;
      h->info.d_probe[p] = 0;
    }
    if (!(norm1 > 0.0)) break;  // L = 0: every d_p is 0
    E.n = n;
    E.s = s;
    E.fwd.n = n; E.fwd.rp = h->row_ptr; E.fwd.col = h->col; E.fwd.val = h->val;
    set_wave(E.fwd, h);
    E.fsplit = h->split;
    if (adj_fwd) {
      E.adj = E.fwd;
      E.adj.adj_fwd = 1;
      E.adj.trp = dtrp;
      E.adj.tcol = dtcol;
      E.adj.tval = dtval;
      E.asplit = true;
    } else {
      // adjoint wave-jagged layout (transient)
      if ((e = build_wave_layout(arp, acol, aval, n, annz, N, s, WA)) != hipSuccess) break;
      E.adj.n = n; E.adj.rp = arp; E.adj.col = acol; E.adj.val = aval;
      set_wave(E.adj, WA);
      E.adj.N = N;
      E.asplit = WA.split;
    }
    E.grid = wave_grid(h->nwb, resident_workgroups(1));
    if ((e = dalloc(&E.X, 2 * (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.Y, 2 * (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.W0, 2 * (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.W1, 2 * (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.S, 2 * (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.h, (size_t)n)) != hipSuccess) break;
    if ((e = dalloc(&E.part, 2 * (size_t)E.grid)) != hipSuccess) break;
    if ((e = dalloc(&E.sums, 2)) != hipSuccess) break;
    if ((e = dalloc(&E.cand_v, (size_t)E.grid * kTopKMax)) != hipSuccess) break;
    if ((e = dalloc(&E.cand_i, (size_t)E.grid * kTopKMax)) != hipSuccess) break;
    if ((e = dalloc(&E.top_v, kTopKMax)) != hipSuccess) break;
    if ((e = dalloc(&E.top_i, kTopKMax)) != hipSuccess) break;
    if ((e = dalloc(&E.first_sums, 2 * (kPMax + 2))) != hipSuccess) break;
    for (int p = 2; p <= kPMax + 1 && e == hipSuccess; ++p) e = dalloc(&E.Sp[p], 2 * (size_t)n);
    if (e == hipSuccess) e = post_get(&E.post_host, &E.post_dev);
    if (e == hipSuccess) E.post_seq = __atomic_load_n(&E.post_host->seq, __ATOMIC_ACQUIRE);
    if (e != hipSuccess) break;
    // Chains merged per matrix pass (QSW_EST_CHAINS; 1: one estimate at a
    // time).  By default only for operators of at most kEstMergeMaxN rows:
    // there the launches and host round trips they save dominate (N = 256:
    // build 2.87 -> 2.52 ms), while on larger ones the wide blocks' gathers,
    // unstaged and many columns wide, cost more than the passes they save
    // (N = 1024: 21.1 -> 36.3 ms).
    const int dflt = n <= kEstMergeMaxN ? kEstChainsMax : 1;
    E.width = std::min(kEstChainsMax, std::max(1, env_int("QSW_EST_CHAINS", dflt)));
    E.width = (int)std::min<int64_t>(E.width, (int64_t)(kEstWideBytes / (2 * sizeof(double2) * (size_t)n)));
    if (n < 2) E.width = 1;
    if (E.width >= 2) {
      const size_t wide = 2 * (size_t)E.width * (size_t)n;
      if ((e = dalloc(&E.Win, wide)) != hipSuccess) break;
      if ((e = dalloc(&E.Wa, wide)) != hipSuccess) break;
      if ((e = dalloc(&E.Wb, wide)) != hipSuccess) break;
      if ((e = dalloc(&E.hc, (size_t)E.width * (size_t)n)) != hipSuccess) break;
      if ((e = dalloc(&E.partc, (size_t)E.width * 2 * (size_t)E.grid)) != hipSuccess) break;
      if ((e = dalloc(&E.sumc, 2 * (size_t)E.width)) != hipSuccess) break;
      if ((e = dalloc(&E.topc_v, (size_t)E.width * kTopKMax)) != hipSuccess) break;
      if ((e = dalloc(&E.topc_i, (size_t)E.width * kTopKMax)) != hipSuccess) break;
    }
    if ((e = E.first_pass(kPMax + 1)) != hipSuccess) break;
    if (E.width >= 2) {
      // groups of `width` estimates, largest p first
      for (int top = kPMax + 1; top >= 2 && e == hipSuccess;) {
        std::vector<int> ps;
        for (int p = top; p >= 2 && (int)ps.size() < E.width; --p) ps.push_back(p);
        top -= (int)ps.size();
        double est[kEstChainsMax];
        int64_t idx[kEstChainsMax];
        int probe[kEstChainsMax];
        if ((e = E.estimate_merged(ps, est, idx, probe)) != hipSuccess) break;
        for (size_t j = 0; j < ps.size(); ++j) {
          h->info.d[ps[j]] = std::pow(est[j], 1.0 / ps[j]);
          h->info.d_index[ps[j]] = idx[j];
          h->info.d_probe[ps[j]] = probe[j];
        }
      }
      if (e != hipSuccess) break;
    } else {
      // one estimate at a time, largest p first (unit-column chains kept
      // for the later ones when the memory allows)
      const size_t lad_bytes = (size_t)kPMax * 2 * sizeof(double2) * (size_t)n;
      if (env_int("QSW_EST_SHARE", 1) != 0 && lad_bytes <= kEstWideBytes) {
        for (int q = 1; q <= kPMax && e == hipSuccess; ++q) e = dalloc(&E.lad[q], 2 * (size_t)n);
        if (e != hipSuccess) {
          // an optimisation only: without the memory, no chains are kept
          (void)hipGetLastError();
          for (double2 *&b : E.lad) dfree(b);
          e = hipSuccess;
        }
      }
      for (int p = kPMax + 1; p >= 2; --p) {
        double est = 0.0;
        int64_t idx = -1;
        int probe = 0;
        if ((e = E.estimate(p, &est, &idx, &probe)) != hipSuccess) break;
        h->info.d[p] = std::pow(est, 1.0 / p);
        h->info.d_index[p] = idx;
        h->info.d_probe[p] = probe;
      }
    }
  } while (false);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(nbits);
  WA.release();
  dfree(E.X); dfree(E.Y); dfree(E.W0); dfree(E.W1); dfree(E.S); dfree(E.h); dfree(E.part); dfree(E.sums);
  dfree(E.cand_v); dfree(E.cand_i); dfree(E.top_v); dfree(E.top_i);
  dfree(E.first_sums);
  dfree(E.Win); dfree(E.Wa); dfree(E.Wb); dfree(E.hc); dfree(E.partc); dfree(E.sumc);
  dfree(E.topc_v); dfree(E.topc_i);
  for (double2 *&b : E.Sp) dfree(b);
  for (double2 *&b : E.lad) dfree(b);
  // back to the pool only with no post in flight (else it is left allocated)
  if (e == hipSuccess || hipStreamSynchronize(s) == hipSuccess) post_put(E.post_host, E.post_dev);
  dfree(arp); dfree(acol); dfree(aval);
  dfree(dfrp); dfree(dtrp); dfree(dtcol); dfree(dtval);
  if (e != hipSuccess) return fail(status_of(e));
  if (!std::isfinite(norm1)) return fail(QSW_ERR_NONFINITE);
  h->info.N = N;
  h->info.n = n;
  h->info.nnz = h->nnz;
  h->info.omega = omega;
  h->info.norm_products = E.products;
  h->info.split = h->split ? 1 : 0;
  h->info.stream_entries = h->wentries;
  h->info.shared_entries = h->wshared;
  h->info.distinct_entries = h->wdistinct;
  if (hipEventCreate(&h->ev_start) != hipSuccess || hipEventCreate(&h->ev_end) != hipSuccess)
    return fail(QSW_ERR_DEVICE);
  if (dalloc(&h->stats_dev, 3) != hipSuccess) return fail(QSW_ERR_OOM);
  auto t_end = std::chrono::steady_clock::now();
  h->info.build_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
  *out = h;
  return QSW_OK;
}

}  // namespace

// ------------------------------------------------------------ propagate plan

qsw_status_t qsw::make_plan(const qsw_superop_s *h, double t0, double dt, int32_t n_steps,
                             Plan &P) {
  if (!std::isfinite(t0) || !std::isfinite(dt) || n_steps < 0) return QSW_ERR_ARG;
  // The handle's d_p were estimated at construction (the paper computes the
  // 1-norm series once, Section 4 footnote), so the alpha_p rule decides for
  // every t: Al-Mohy and Higham's switch to the 1-norm rule for small
  // ||tL||_1 only saves the products of estimating them.
  const double *d = h->info.d;
  qsw_status_t st;
  if (t0 != 0.0) {
    st = select_params_impl(h->info.norm1, d, t0, 1, h->prec, &P.m0, &P.s0, false);
    if (st != QSW_OK) return st;
  }
  const size_t vec = (size_t)h->n * sizeof(double2);
  P.off_state = 0;
  size_t off = align256(sizeof(DeviceState));
  if (h->prec == QSW_PREC_FP32) {
    // single-precision products: one single-time application per interval;
    // two complex64 terms, two hi + lo accumulator pairs
    if (n_steps > 0) {
      st = select_params_impl(h->info.norm1, d, dt, 1, h->prec, &P.m, &P.s, false);
      if (st != QSW_OK) return st;
    }
    const size_t v32 = align256((size_t)h->n * sizeof(float2));
    P.branch = 0;
    P.off_pts = off;
    P.off_B = off;
    off += 2 * v32;
    P.off_F = off;
    off += 4 * v32;
    P.off_K = off;
    P.total = off;
    return QSW_OK;
  }
  if (n_steps > 0) {
    int mS = 0, sS = 1;
    st = select_params_impl(h->info.norm1, d, (double)n_steps * dt, 1, h->prec, &mS, &sS, false);
    if (st != QSW_OK) return st;
    if (n_steps <= sS || mS == 0) {
      P.branch = 0;
      st = select_params_impl(h->info.norm1, d, dt, 1, h->prec, &P.m, &P.s, false);
      if (st != QSW_OK) return st;
    } else {
      P.branch = 1;
      P.m = mS;
      P.s = sS;
      P.d = n_steps / sS;
      P.j = n_steps / P.d;
      P.r = n_steps - P.d * P.j;
    }
  }
  P.off_pts = off;
  if (P.branch == 1) off += align256(sizeof(PointSlots) * (size_t)P.d);
  P.off_B = off;
  off += 2 * align256(vec);
  P.off_F = off;
  off += 2 * align256(vec);
  P.off_K = off;
  if (P.branch == 1) off += (size_t)P.m * align256(vec);
  P.total = off;
  return QSW_OK;
}

namespace {

struct Runner {
  qsw_superop_s *h;
  hipStream_t s;
  DeviceState *st;
  double2 *B[2];
  double2 *F[2];
  int64_t gstep = 0;
  int64_t launched = 0;
  double tol;
  int engine;  // product engine of this call (value format included)
  // paced term launches (null pace_dev: not paced)
  unsigned long long *pace_dev = nullptr;
  unsigned long long *pace_host = nullptr;
  unsigned long long *seq = nullptr;
  int pace = 0;
  // launches up to `retired` count as finished: those of earlier calls and
  // those of a step that has passed its test (they exit at once)
  unsigned long long retired = 0;

  // Waits until launch number `next` is at most `pace` launches ahead of the
  // last launch known to have ended (each term launch posts its predecessor);
  // returns true instead once the step whose first launch was `first` has
  // passed its test (its remaining terms would exit at once).  Stops waiting
  // when the stream has drained, as no further word can arrive then.
  //
  // With a lookahead of 1 only the drain shows that the last launch has
  // ended, so the stream is queried all along.  With more, a later launch
  // already in the stream posts the word, and the query only guards against
  // a stream that stopped (a device error): it is made after 10 ms.  A query
  // puts a marker behind the running kernel, which delays the next launch by
  // about 6 us; made while every launch waits, it cost 8 ms per benchmark pass.
  bool wait_paced(unsigned long long next, unsigned long long first) {
    using clock = std::chrono::steady_clock;
    const auto every = std::chrono::milliseconds(pace == 1 ? 0 : 10);
    auto query_at = clock::now() + every;
    for (unsigned spins = 1;; ++spins) {
      const unsigned long long w = __atomic_load_n(pace_host, __ATOMIC_ACQUIRE);
      const unsigned long long done = w >> 1;
      if ((w & 1ull) && done >= first) {
        retired = std::max(retired, next - 1);
        return true;
      }
      if (next <= std::max(done, retired) + (unsigned long long)pace) return false;
      if ((spins & 1023u) == 0) {
        const auto now = clock::now();
        if (now >= query_at) {
          if (hipStreamQuery(s) != hipErrorNotReady) return false;
          query_at = now + every;
        }
      }
    }
  }

  SpmvArgs base_args() const {
    SpmvArgs a{};
    a.n = h->n;
    a.rp = h->row_ptr;
    a.col = h->col;
    a.val = h->val;
    a.tol = tol;
    a.st = st;
    a.rows_per_block = h->rows_per_block;
    a.blk = h->blk;
    a.nblk = h->nblk;
    a.blocks_per_wg = h->blocks_per_wg;
    set_wave(a, h);
    return a;
  }

  // Single-precision products: complex64 terms B32 and the hi + lo
  // accumulator pairs (Fh[c], Fl[c]); the state is pair `cur`.
  float2 *B32[2] = {nullptr, nullptr};
  float2 *Fh[2] = {nullptr, nullptr}, *Fl[2] = {nullptr, nullptr};
  int cur = 0;

  // State = T_m(t L / s)^s state, terms in single precision (the stopping
  // test and the sums of the norms as in alg32).
  hipError_t alg32_f32(double t, int m, int s_steps) {
    if (m == 0) return hipSuccess;
    for (int i = 0; i < s_steps; ++i) {
      const int par = (int)(gstep & 1);
      ++gstep;
      const int src = cur, dst = cur ^ 1;
      const unsigned long long first = seq ? *seq + 1 : 0;
      for (int j = 1; j <= m; ++j) {
        SpmvArgs a = base_args();
        if (pace_dev) {
          if (wait_paced(*seq + 1, first)) break;
          a.progress = pace_dev;
          a.seq = ++*seq;
        }
        // term 1 multiplies the state's hi part (the state rounded to float)
        a.x32 = (j == 1) ? Fh[src] : B32[(j - 1) & 1];
        a.y32 = B32[j & 1];
        a.fin_hi = (j == 1) ? Fh[src] : Fh[dst];
        a.fin_lo = (j == 1) ? Fl[src] : Fl[dst];
        a.fout_hi = Fh[dst];
        a.fout_lo = Fl[dst];
        a.alpha = t / ((double)s_steps * (double)j);
        a.par = par;
        a.j = j;
        hipError_t e = launch_taylor_term32(a, engine, h->grid, s);
        if (e != hipSuccess) return e;
        ++launched;
      }
      cur = dst;
    }
    return hipSuccess;
  }

  // x_out = T_m(t L / s)^s x_in with the early-termination test on the device.
  hipError_t alg32(const double2 *x_in, double2 *x_out, double t, int m, int s_steps) {
    if (m == 0) return launch_copy(x_out, x_in, h->n, s);
    const double2 *Fsrc = x_in;
    for (int i = 0; i < s_steps; ++i) {
      const int par = (int)(gstep & 1);
      ++gstep;
      double2 *Fdst = (i == s_steps - 1) ? x_out : F[i & 1];
      const unsigned long long first = seq ? *seq + 1 : 0;
      for (int j = 1; j <= m; ++j) {
        SpmvArgs a = base_args();
        if (pace_dev) {
          if (wait_paced(*seq + 1, first)) break;
          a.progress = pace_dev;
          a.seq = ++*seq;
        }
        a.x = (j == 1) ? Fsrc : B[(j - 1) & 1];
        a.y = B[j & 1];
        a.fin = (j == 1) ? Fsrc : Fdst;
        a.fout = Fdst;
        a.alpha = t / ((double)s_steps * (double)j);
        a.par = par;
        a.j = j;
        hipError_t e = launch_taylor_term(a, engine, h->grid, s);
        if (e != hipSuccess) return e;
        ++launched;
      }
      Fsrc = Fdst;
    }
    return hipSuccess;
  }
};

}  // namespace

// ================================================================== C ABI

extern "C" {

const char *qsw_status_str(qsw_status_t s) {
  switch (s) {
    case QSW_OK: return "ok";
    case QSW_ERR_ARG: return "invalid argument";
    case QSW_ERR_GRAPH: return "malformed graph or operator CSR";
    case QSW_ERR_OOM: return "device out of memory";
    case QSW_ERR_DEVICE: return "HIP runtime error";
    case QSW_ERR_NONFINITE: return "non-finite value";
    case QSW_ERR_STATE: return "bad state (device, workspace)";
    case QSW_ERR_SIZE: return "N*N exceeds the 32-bit column index";
    case QSW_ERR_SCRATCH:
      return "the propagation needs more than the static scratch of qsw_propagate_noalloc";
  }
  return "unknown status";
}

const char *qsw_version(void) { return "qsw 0.1 gfx950"; }

}  // extern "C"

namespace {

struct Pool {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void *>> kept;   // (device, bytes) -> blocks
  std::unordered_map<void *, std::pair<int, size_t>> live;      // allocated blocks
  size_t held = 0;                                               // bytes kept
  size_t cap = 0;
  Pool() { cap = (size_t)std::max(0, env_int("QSW_POOL_MB", 16384)) << 20; }
  void release_device(int dev) {  // mu held; `dev` current
    for (auto it = kept.begin(); it != kept.end();) {
      if (it->first.first != dev) {
        ++it;
        continue;
      }
      for (void *b : it->second) {
        (void)hipFree(b);
        held -= it->first.second;
      }
      it = kept.erase(it);
    }
  }
};

Pool &pool() {
  static Pool *p = new Pool();  // kept until the process ends
  return *p;
}

}  // namespace

hipError_t qsw::pool_alloc(void **p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Pool &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.kept.find({dev, bytes});
  if (it != P.kept.end() && !it->second.empty()) {
    *p = it->second.back();
    it->second.pop_back();
    P.held -= bytes;
  } else {
    e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory && P.held > 0) {
      (void)hipGetLastError();
      P.release_device(dev);
      e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
      *p = nullptr;
      return e;
    }
  }
  P.live[*p] = {dev, bytes};
  return hipSuccess;
}

void qsw::pool_free(void *p) {
  if (!p) return;
  Pool &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) {  // not from pool_alloc
    (void)hipFree(p);
    return;
  }
  const int dev = it->second.first;
  const size_t bytes = it->second.second;
  P.live.erase(it);
  DeviceGuard g(dev);
  if (g.ok && P.held + bytes <= P.cap && hipDeviceSynchronize() == hipSuccess) {
    P.kept[{dev, bytes}].push_back(p);
    P.held += bytes;
  } else {
    (void)hipFree(p);
  }
}

namespace {

// Operators of a walk on a graph (Section 2.5.1): H from G^u, rates from G
// (eq. generator_matrix, eq. lindblad), as the flags select.
qsw_status_t graph_ops(int32_t N, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
                       double gamma, uint32_t flags, HostOps &op) {
  const int64_t E = row_ptr[N];
  if (E > 0 && (!col_idx || !w)) return QSW_ERR_ARG;
  qsw_status_t st = check_csr(N, row_ptr, col_idx, false);
  if (st != QSW_OK) return st;
  for (int64_t e = 0; e < E; ++e)
    if (!(w[e] > 0.0) || !std::isfinite(w[e])) return QSW_ERR_GRAPH;
  // G^u = max(G, G^T) by merging each row of G with the same row of G^T
  std::vector<int64_t> gp(row_ptr, row_ptr + N + 1), tp;
  std::vector<int32_t> gc(col_idx, col_idx + E), tc;
  std::vector<double> gw(w, w + E), tw;
  transpose_csr(N, gp, gc, gw, 1, tp, tc, tw);
  op.N = N;
  op.hp.assign(N + 1, 0);
  op.hdiag.assign(N, 0.0);
  std::vector<int32_t> uc;
  std::vector<double> uw;
  uc.reserve(2 * E);
  uw.reserve(2 * E);
  for (int32_t i = 0; i < N; ++i) {
    int64_t a = gp[i], b = tp[i];
    while (a < gp[i + 1] || b < tp[i + 1]) {
      const int32_t ca = a < gp[i + 1] ? gc[a] : INT32_MAX;
      const int32_t cb = b < tp[i + 1] ? tc[b] : INT32_MAX;
      if (ca == cb) {
        uc.push_back(ca);
        uw.push_back(std::max(gw[a], tw[b]));
        ++a;
        ++b;
      } else if (ca < cb) {
        uc.push_back(ca);
        uw.push_back(gw[a++]);
      } else {
        uc.push_back(cb);
        uw.push_back(tw[b++]);
      }
    }
    op.hp[i + 1] = (int64_t)uc.size();
  }
  const bool laplacian = !(flags & QSW_H_ADJACENCY);
  op.hc = uc;
  op.hv.assign(2 * uc.size(), 0.0);
  for (int32_t i = 0; i < N; ++i) {
    double deg = 0.0;
    for (int64_t e = op.hp[i]; e < op.hp[i + 1]; ++e) {
      deg += uw[e];
      op.hv[2 * e] = laplacian ? -gamma * uw[e] : uw[e];
    }
    op.hdiag[i] = laplacian ? gamma * deg : 0.0;
  }
  // rates: R_ij for each arc j -> i (row i of G), plus optional dephasing
  std::vector<double> outdeg(N, 0.0);
  for (int64_t e = 0; e < E; ++e) outdeg[gc[e]] += gw[e];
  const bool colnorm = (flags & QSW_R_COLNORM) != 0;
  op.rp = gp;
  op.rc = gc;
  op.rv.resize(E);
  for (int64_t e = 0; e < E; ++e) op.rv[e] = colnorm ? gw[e] / outdeg[gc[e]] : gamma * gw[e];
  op.rdiag.assign(N, 0.0);
  if (flags & QSW_DEPHASING)
    for (int32_t j = 0; j < N; ++j)
      op.rdiag[j] = colnorm ? (outdeg[j] > 0.0 ? 1.0 : 0.0) : gamma * outdeg[j];
  return QSW_OK;
}

}  // namespace

extern "C" {

qsw_status_t qsw_superop_build(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                               const double *w, double omega, double gamma, uint32_t flags,
                               void *hip_stream, qsw_superop_t *out) {
  return qsw_superop_build_channels(N, row_ptr, col_idx, w, omega, gamma, flags, 0, nullptr,
                                    nullptr, 0, nullptr, nullptr, hip_stream, out);
}

qsw_status_t qsw_superop_build_channels(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                                        const double *w, double omega, double gamma,
                                        uint32_t flags, int32_t n_sources,
                                        const int32_t *source_vertex, const double *source_rate,
                                        int32_t n_sinks, const int32_t *sink_vertex,
                                        const double *sink_rate, void *hip_stream,
                                        qsw_superop_t *out) {
  if (!out || !row_ptr || N < 1 || n_sources < 0 || n_sinks < 0) return QSW_ERR_ARG;
  *out = nullptr;
  if (!(omega >= 0.0 && omega <= 1.0) || !(gamma > 0.0) || !std::isfinite(gamma)) return QSW_ERR_ARG;
  if (flags & ~(uint32_t)(QSW_H_ADJACENCY | QSW_R_COLNORM | QSW_DEPHASING)) return QSW_ERR_ARG;
  if ((n_sources > 0 && (!source_vertex || !source_rate)) ||
      (n_sinks > 0 && (!sink_vertex || !sink_rate)))
    return QSW_ERR_ARG;
  const int64_t Na = (int64_t)N + n_sources + n_sinks;  // order of the augmented digraph
  if (Na * Na > (int64_t)std::numeric_limits<int32_t>::max()) return QSW_ERR_SIZE;
  if (row_ptr[N] > 0 && (!col_idx || !w)) return QSW_ERR_ARG;
  for (int32_t k = 0; k < n_sources; ++k)
    if (source_vertex[k] < 0 || source_vertex[k] >= N || !(source_rate[k] > 0.0) ||
        !std::isfinite(source_rate[k]))
      return QSW_ERR_GRAPH;
  for (int32_t k = 0; k < n_sinks; ++k)
    if (sink_vertex[k] < 0 || sink_vertex[k] >= N || !(sink_rate[k] > 0.0) ||
        !std::isfinite(sink_rate[k]))
      return QSW_ERR_GRAPH;
  HostOps op;
  qsw_status_t st = graph_ops(N, row_ptr, col_idx, w, gamma, flags, op);
  if (st != QSW_OK) return st;
  if (Na > N) {
    // the augmented digraph: source k is vertex N + k, sink k is vertex
    // N + n_sources + k; H and the omega rates are zero on them, and the
    // channels are rates outside omega (eq. qsw_ss)
    const int32_t M = (int32_t)Na;
    op.N = M;
    op.hp.resize(M + 1, op.hp[N]);
    op.hdiag.resize(M, 0.0);
    op.rp.resize(M + 1, op.rp[N]);
    op.rdiag.resize(M, 0.0);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(M);
    for (int32_t k = 0; k < n_sources; ++k)  // source N + k -> vertex
      rows[source_vertex[k]].push_back({N + k, source_rate[k]});
    for (int32_t k = 0; k < n_sinks; ++k)  // vertex -> sink N + n_sources + k
      rows[N + n_sources + k].push_back({sink_vertex[k], sink_rate[k]});
    op.fp.assign(M + 1, 0);
    op.fdiag.assign(M, 0.0);
    for (int32_t i = 0; i < M; ++i) {
      std::sort(rows[i].begin(), rows[i].end());
      for (size_t t = 0; t < rows[i].size(); ++t) {
        if (t > 0 && rows[i][t].first == rows[i][t - 1].first) {
          op.fv.back() += rows[i][t].second;  // two channels on one arc add up
          continue;
        }
        op.fc.push_back(rows[i][t].first);
        op.fv.push_back(rows[i][t].second);
      }
      op.fp[i + 1] = (int64_t)op.fc.size();
    }
  }
  auto src = std::make_shared<LocalAssembler>();
  src->op = std::move(op);
  return build_common(src, omega, (hipStream_t)hip_stream, out);
}

qsw_status_t qsw_superop_build_ops(int32_t N, const int64_t *h_row_ptr, const int32_t *h_col,
                                   const double *h_val, const int64_t *l_row_ptr,
                                   const int32_t *l_col, const double *l_val, double omega,
                                   uint32_t flags, void *hip_stream, qsw_superop_t *out) {
  return qsw_superop_build_open(N, h_row_ptr, h_col, h_val, l_row_ptr, l_col, l_val, nullptr,
                                nullptr, nullptr, omega, flags, hip_stream, out);
}

qsw_status_t qsw_superop_build_open(int32_t N, const int64_t *h_row_ptr, const int32_t *h_col,
                                    const double *h_val, const int64_t *l_row_ptr,
                                    const int32_t *l_col, const double *l_val,
                                    const int64_t *f_row_ptr, const int32_t *f_col,
                                    const double *f_val, double omega, uint32_t flags,
                                    void *hip_stream, qsw_superop_t *out) {
  if (!out || !h_row_ptr || !l_row_ptr || N < 1) return QSW_ERR_ARG;
  *out = nullptr;
  if (!(omega >= 0.0 && omega <= 1.0) || flags != 0) return QSW_ERR_ARG;
  if ((int64_t)N * N > (int64_t)std::numeric_limits<int32_t>::max()) return QSW_ERR_SIZE;
  HostOps op;
  op.N = N;
  qsw_status_t st = parse_hermitian(N, h_row_ptr, h_col, h_val, op);
  if (st != QSW_OK) return st;
  st = parse_rates(N, l_row_ptr, l_col, l_val, op.rp, op.rc, op.rv, op.rdiag);
  if (st != QSW_OK) return st;
  if (f_row_ptr) {
    st = parse_rates(N, f_row_ptr, f_col, f_val, op.fp, op.fc, op.fv, op.fdiag);
    if (st != QSW_OK) return st;
  }
  auto src = std::make_shared<LocalAssembler>();
  src->op = std::move(op);
  return build_common(src, omega, (hipStream_t)hip_stream, out);
}

qsw_status_t qsw_superop_build_general(int32_t N, const int64_t *h_row_ptr, const int32_t *h_col,
                                       const double *h_val, int32_t n_ops,
                                       const int64_t *const *l_row_ptr,
                                       const int32_t *const *l_col, const double *const *l_val,
                                       const int64_t *r_row_ptr, const int32_t *r_col,
                                       const double *r_val, double omega, void *hip_stream,
                                       qsw_superop_t *out) {
  if (!out || !h_row_ptr || N < 1 || n_ops < 0 || (n_ops > 0 && (!l_row_ptr || !l_col || !l_val)))
    return QSW_ERR_ARG;
  *out = nullptr;
  if (!(omega >= 0.0 && omega <= 1.0)) return QSW_ERR_ARG;
  if ((int64_t)N * N > (int64_t)std::numeric_limits<int32_t>::max()) return QSW_ERR_SIZE;
  auto src = std::make_shared<GeneralAssembler>();
  src->N = N;
  qsw_status_t st = parse_complex(N, h_row_ptr, h_col, h_val, true, src->H);
  if (st != QSW_OK) return st;
  if (r_row_ptr) {
    st = parse_complex(N, r_row_ptr, r_col, r_val, true, src->Hrot);
    if (st != QSW_OK) return st;
  }
  for (int32_t k = 0; k < n_ops; ++k) {
    HostCsr L;
    st = parse_complex(N, l_row_ptr[k], l_col[k], l_val[k], false, L);
    if (st != QSW_OK) return st;
    src->LdLs.push_back(product(N, conj_transpose(N, L), L));
    src->Ls.push_back(std::move(L));
  }
  return build_common(src, omega, (hipStream_t)hip_stream, out);
}

int32_t qsw_demoralised_order(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                              int32_t *copies) {
  if (!row_ptr || N < 1 || (row_ptr[N] > 0 && !col_idx)) return -1;
  if (check_csr(N, row_ptr, col_idx, false) != QSW_OK) return -1;
  int64_t M = 0;
  for (int32_t v = 0; v < N; ++v) {
    const int64_t d = std::max<int64_t>(1, row_ptr[v + 1] - row_ptr[v]);  // parents of v
    if (copies) copies[v] = (int32_t)d;
    M += d;
  }
  return M > std::numeric_limits<int32_t>::max() ? -1 : (int32_t)M;
}

qsw_status_t qsw_superop_build_demoralised(int32_t N, const int64_t *row_ptr,
                                           const int32_t *col_idx, const double *w, double omega,
                                           double gamma, void *hip_stream, qsw_superop_t *out) {
  if (!out || !row_ptr || N < 1) return QSW_ERR_ARG;
  *out = nullptr;
  if (!(omega >= 0.0 && omega <= 1.0) || !(gamma > 0.0) || !std::isfinite(gamma)) return QSW_ERR_ARG;
  const int64_t E = row_ptr[N];
  if (E > 0 && (!col_idx || !w)) return QSW_ERR_ARG;
  qsw_status_t st = check_csr(N, row_ptr, col_idx, false);
  if (st != QSW_OK) return st;
  for (int64_t e = 0; e < E; ++e)
    if (!(w[e] > 0.0) || !std::isfinite(w[e])) return QSW_ERR_GRAPH;
  std::vector<int32_t> d(N);
  const int32_t M = qsw_demoralised_order(N, row_ptr, col_idx, d.data());
  if (M < 0) return QSW_ERR_SIZE;
  if ((int64_t)M * M > (int64_t)std::numeric_limits<int32_t>::max()) return QSW_ERR_SIZE;
  std::vector<int64_t> off(N + 1, 0);
  for (int32_t v = 0; v < N; ++v) off[v + 1] = off[v] + d[v];
  // G^u = max(G, G^T)
  std::vector<int64_t> gp(row_ptr, row_ptr + N + 1), tp;
  std::vector<int32_t> gc(col_idx, col_idx + E), tc;
  std::vector<double> gw(w, w + E), tw;
  transpose_csr(N, gp, gc, gw, 1, tp, tc, tw);
  std::vector<std::vector<std::pair<int32_t, double>>> urow(N);
  for (int32_t v = 0; v < N; ++v) {
    int64_t a = gp[v], b = tp[v];
    while (a < gp[v + 1] || b < tp[v + 1]) {
      const int32_t ca = a < gp[v + 1] ? gc[a] : INT32_MAX;
      const int32_t cb = b < tp[v + 1] ? tc[b] : INT32_MAX;
      if (ca == cb) {
        urow[v].push_back({ca, std::max(gw[a++], tw[b++])});
      } else if (ca < cb) {
        urow[v].push_back({ca, gw[a++]});
      } else {
        urow[v].push_back({cb, tw[b++]});
      }
    }
  }
  auto src = std::make_shared<GeneralAssembler>();
  src->N = M;
  // H_D: transition matrix (eq. generator_matrix) of the demoralised graph,
  // copies joined with weight G^u_vw / sqrt(d_v d_w) (eq. nm_weight)
  {
    std::vector<std::vector<std::pair<int32_t, std::complex<double>>>> rows(M);
    std::vector<double> deg(M, 0.0);
    for (int32_t v = 0; v < N; ++v)
      for (const auto &[u, gu] : urow[v]) {
        const double wd = gu / std::sqrt((double)d[v] * d[u]);
        for (int32_t k = 0; k < d[v]; ++k)
          for (int32_t l = 0; l < d[u]; ++l) {
            rows[off[v] + k].push_back({(int32_t)(off[u] + l), -gamma * wd});
            deg[off[u] + l] += wd;
          }
      }
    for (int32_t i = 0; i < M; ++i) rows[i].push_back({i, gamma * deg[i]});
    HostCsr &H = src->H;
    H.rp.assign(M + 1, 0);
    for (int32_t i = 0; i < M; ++i) {
      std::sort(rows[i].begin(), rows[i].end(),
                [](const auto &x, const auto &y) { return x.first < y.first; });
      for (const auto &e : rows[i]) {
        H.col.push_back(e.first);
        H.val.push_back(e.second);
      }
      H.rp[i + 1] = (int64_t)H.col.size();
    }
  }
  // L_D (eq. dm_lind): copy u of parent w of v -> copy k of v with
  // F_v[k][m] G_vw / sqrt(d_v d_w), m the rank of w among v's parents and F_v
  // the Fourier matrix exp(2 pi i k m / d_v) with unit-modulus entries
  {
    const double pi = std::acos(-1.0);
    std::vector<std::vector<std::pair<int32_t, std::complex<double>>>> rows(M);
    for (int32_t v = 0; v < N; ++v)
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int32_t wv = col_idx[e];
        const int32_t m = (int32_t)(e - row_ptr[v]);
        const double g = w[e] / std::sqrt((double)d[v] * d[wv]);
        for (int32_t k = 0; k < d[v]; ++k) {
          const double ang = 2.0 * pi * (double)((int64_t)k * m % d[v]) / (double)d[v];
          const std::complex<double> f(std::cos(ang), std::sin(ang));
          for (int32_t u = 0; u < d[wv]; ++u) rows[off[v] + k].push_back({(int32_t)(off[wv] + u), f * g});
        }
      }
    HostCsr L;
    L.rp.assign(M + 1, 0);
    for (int32_t i = 0; i < M; ++i) {
      std::sort(rows[i].begin(), rows[i].end(),
                [](const auto &x, const auto &y) { return x.first < y.first; });
      for (const auto &e : rows[i]) {
        L.col.push_back(e.first);
        L.val.push_back(e.second);
      }
      L.rp[i + 1] = (int64_t)L.col.size();
    }
    src->LdLs.push_back(product(M, conj_transpose(M, L), L));
    src->Ls.push_back(std::move(L));
  }
  // H_rot (eq. H_rot): +i from copy k to copy k+1 of one vertex, -i back;
  // cyclic (k = d-1 to 0) when d > 2
  {
    std::vector<std::vector<std::pair<int32_t, std::complex<double>>>> rows(M);
    bool any = false;
    for (int32_t v = 0; v < N; ++v) {
      if (d[v] < 2) continue;
      any = true;
      for (int32_t k = 0; k < d[v]; ++k) {
        const int32_t l = (k + 1) % d[v];
        if (d[v] == 2 && k == 1) break;  // the single pair of two copies
        rows[off[v] + l].push_back({(int32_t)(off[v] + k), std::complex<double>(0.0, 1.0)});
        rows[off[v] + k].push_back({(int32_t)(off[v] + l), std::complex<double>(0.0, -1.0)});
      }
    }
    if (any) {
      HostCsr &R = src->Hrot;
      R.rp.assign(M + 1, 0);
      for (int32_t i = 0; i < M; ++i) {
        std::sort(rows[i].begin(), rows[i].end(),
                  [](const auto &x, const auto &y) { return x.first < y.first; });
        for (const auto &e : rows[i]) {
          R.col.push_back(e.first);
          R.val.push_back(e.second);
        }
        R.rp[i + 1] = (int64_t)R.col.size();
      }
    }
  }
  return build_common(src, omega, (hipStream_t)hip_stream, out);
}

qsw_status_t qsw_demoralised_state(int32_t N, const int32_t *copies, const double *rho,
                                   double *rho_d) {
  if (!copies || !rho || !rho_d || N < 1) return QSW_ERR_ARG;
  std::vector<int64_t> off(N + 1, 0);
  for (int32_t v = 0; v < N; ++v) {
    if (copies[v] < 1) return QSW_ERR_ARG;
    off[v + 1] = off[v] + copies[v];
  }
  const int64_t M = off[N];
  for (int32_t a = 0; a < N; ++a)
    for (int32_t b = 0; b < N; ++b) {
      const double f = 1.0 / std::sqrt((double)copies[a] * copies[b]);
      const double re = rho[2 * ((int64_t)a * N + b)] * f, im = rho[2 * ((int64_t)a * N + b) + 1] * f;
      for (int64_t i = off[a]; i < off[a + 1]; ++i)
        for (int64_t j = off[b]; j < off[b + 1]; ++j) {
          rho_d[2 * (i * M + j)] = re;
          rho_d[2 * (i * M + j) + 1] = im;
        }
    }
  return QSW_OK;
}

qsw_status_t qsw_demoralised_populations(int32_t N, const int32_t *copies, const double *pops_d,
                                         int32_t count, double *pops) {
  if (!copies || !pops_d || !pops || N < 1 || count < 0) return QSW_ERR_ARG;
  int64_t M = 0;
  for (int32_t v = 0; v < N; ++v) {
    if (copies[v] < 1) return QSW_ERR_ARG;
    M += copies[v];
  }
  for (int32_t t = 0; t < count; ++t) {
    int64_t i = 0;
    for (int32_t v = 0; v < N; ++v) {
      double p = 0.0;
      for (int32_t k = 0; k < copies[v]; ++k) p += pops_d[t * M + i++];
      pops[(int64_t)t * N + v] = p;
    }
  }
  return QSW_OK;
}

qsw_status_t qsw_superop_set_omega(qsw_superop_t h, double omega, void *hip_stream) {
  if (!h || !h->src) return QSW_ERR_ARG;
  if (!(omega >= 0.0 && omega <= 1.0)) return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  HIP_TRY(hipDeviceSynchronize());  // work in flight may still use the old arrays
  qsw_superop_t nh = nullptr;
  qsw_status_t st = build_common(h->src, omega, (hipStream_t)hip_stream, &nh);
  if (st != QSW_OK) return st;
  const int prec = h->prec;
  // the pacing state stays with the handle
  std::swap(h->pace, nh->pace);
  std::swap(h->pace_host, nh->pace_host);
  std::swap(h->pace_dev, nh->pace_dev);
  std::swap(h->pace_seq, nh->pace_seq);
  std::swap(h->pace_mu, nh->pace_mu);
  std::swap(*h, *nh);
  qsw_superop_destroy(nh);  // the old arrays
  if (prec != QSW_PREC_DOUBLE) return qsw_superop_set_precision(h, prec);
  return QSW_OK;
}

void qsw_superop_destroy(qsw_superop_t h) {
  if (!h) return;
  DeviceGuard g(h->device);
  dfree(h->row_ptr);
  dfree(h->col);
  dfree(h->val);
  dfree(h->stats_dev);
  dfree(h->blk);
  dfree(h->wcol);
  dfree(h->wval);
  dfree(h->wval32);
  dfree(h->wcoef);
  dfree(h->wcoef32);
  dfree(h->wdiag);
  dfree(h->wdiag32);
  dfree(h->wlen);
  dfree(h->wperm);
  dfree(h->wglob);
  dfree(h->wshn);
  dfree(h->wstart);
  dfree(h->wshs);
  dfree(h->wsh);
  if (h->ev_start) (void)hipEventDestroy(h->ev_start);
  if (h->ev_end) (void)hipEventDestroy(h->ev_end);
  if (h->pace_host) (void)hipHostFree(h->pace_host);
  delete h;
}

qsw_status_t qsw_superop_set_precision(qsw_superop_t h, int32_t prec) {
  if (!h || (prec != QSW_PREC_DOUBLE && prec != QSW_PREC_SINGLE && prec != QSW_PREC_FP32))
    return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  const bool have32 = h->split ? h->wcoef32 != nullptr : h->wval32 != nullptr;
  if (prec != QSW_PREC_DOUBLE && !have32) {
    if (!is_wave_engine(h->engine))
      return QSW_ERR_STATE;  // the single-precision copy exists for the wave layout only
    // the padding converts to zeros as well
    hipStream_t s = nullptr;
    const int64_t ent = h->wentries + kWavePad;
    if (h->split) {
      HIP_TRY(dalloc(&h->wcoef32, (size_t)ent));
      HIP_TRY(dalloc(&h->wdiag32, (size_t)h->n));
      HIP_TRY(launch_to_f32(h->wcoef32, h->wcoef, ent, s));
      HIP_TRY(launch_to_c64(h->wdiag32, h->wdiag, h->n, s));
    } else {
      HIP_TRY(dalloc(&h->wval32, (size_t)ent));
      HIP_TRY(launch_to_c64(h->wval32, h->wval, ent, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
  } else if (prec == QSW_PREC_DOUBLE && have32) {
    HIP_TRY(hipDeviceSynchronize());  // earlier calls may still read the copy
    dfree(h->wval32);
    dfree(h->wcoef32);
    dfree(h->wdiag32);
    h->wval32 = nullptr;
    h->wcoef32 = nullptr;
    h->wdiag32 = nullptr;
  }
  h->prec = prec;
  return QSW_OK;
}

qsw_status_t qsw_superop_set_pacing(qsw_superop_t h, int32_t lookahead) {
  if (!h || lookahead < 0 || lookahead > 4096) return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  if (lookahead > 0 && !h->pace_host) {
    void *p = nullptr;
    HIP_TRY(hipHostMalloc(&p, 256, hipHostMallocCoherent));
    h->pace_host = (unsigned long long *)p;
    *h->pace_host = 0ull;
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipHostFree(p);
      h->pace_host = nullptr;
      return QSW_ERR_DEVICE;
    }
    h->pace_dev = (unsigned long long *)d;
    h->pace_seq = 0;
    h->pace_mu.reset(new std::mutex);
  }
  h->pace = lookahead;
  return QSW_OK;
}

qsw_status_t qsw_superop_autotune(qsw_superop_t h, void *hip_stream, qsw_tuning_t *out) {
  if (!h) return QSW_ERR_ARG;
  if (!is_wave_engine(h->engine)) return QSW_ERR_STATE;  // wave-jagged engines only
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  const bool can_stage = (size_t)h->N * sizeof(double2) <= kStageMaxBytes;
  // key: graph order, entries per row (to a quarter), precision, value format
  const long epr = h->n > 0 ? std::lround(4.0 * (double)h->nnz / (double)h->n) : 0;
  const std::tuple<int, long, int, int> key{h->N, epr, h->prec, h->split ? 1 : 0};
  static std::mutex mu;
  static std::map<std::tuple<int, long, int, int>, qsw_tuning_t> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      h->engine = 100 * it->second.staged;
      h->grid = it->second.grid;
      if (out) {
        *out = it->second;
        out->from_cache = 1;
      }
      return QSW_OK;
    }
  }
  double2 *x = nullptr, *y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    dfree(x);
    dfree(y);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (dalloc(&x, (size_t)h->n) != hipSuccess || dalloc(&y, (size_t)h->n) != hipSuccess) {
    cleanup();
    return QSW_ERR_OOM;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      launch_zero(x, (size_t)h->n * sizeof(double2), s) != hipSuccess) {
    cleanup();
    return QSW_ERR_DEVICE;
  }
  const int resident = std::max(resident_workgroups(0), 1);
  qsw_tuning_t best{};
  best.us_per_product = 1e300;
  hipError_t err = hipSuccess;
  // traversals: wide groups (double values), XCD bands, staged, plain
  std::vector<int> trav;
  if (can_stage && h->prec == QSW_PREC_DOUBLE) trav.push_back(3);
  if (can_stage && banded_ok(h->N)) trav.push_back(2);
  if (can_stage) trav.push_back(1);
  trav.push_back(0);
  for (size_t ti = 0; ti < trav.size() && err == hipSuccess; ++ti) {
    const int st = trav[ti];
    for (int mul : {1, 2, 4, 8}) {
      const int64_t wgs = (h->nwb + kBlockThreads / 64 - 1) / (kBlockThreads / 64);
      int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, (int64_t)mul * resident));
      if (st == 2) grid = banded_grid(grid);
      SpmvArgs a{};
      a.n = h->n;
      a.rp = h->row_ptr;
      a.col = h->col;
      a.val = h->val;
      set_wave(a, h);
      a.x = x;
      a.y = y;
      a.alpha = 1.0;
      const int engine = 100 * st + (h->split ? 10 : 0) + (h->prec != QSW_PREC_DOUBLE ? 1 : 0);
      if ((err = launch_spmv(a, engine, grid, s)) != hipSuccess) break;  // warm-up
      if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
      const int reps = 5;
      for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch_spmv(a, engine, grid, s);
      if (err != hipSuccess || (err = hipEventRecord(e1, s)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      const double us = 1e3 * ms / reps;
      if (us < best.us_per_product) {
        best.us_per_product = us;
        best.staged = st;
        best.grid = grid;
      }
      if (wgs <= (int64_t)mul * resident) break;  // larger grids are the same launch
    }
  }
  cleanup();
  if (err != hipSuccess) return status_of(err);
  h->engine = 100 * best.staged;
  h->grid = best.grid;
  {
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
  }
  if (out) *out = best;
  return QSW_OK;
}

qsw_status_t qsw_superop_info(qsw_superop_t h, qsw_info_t *info) {
  if (!h || !info) return QSW_ERR_ARG;
  *info = h->info;
  info->engine = launch_engine(h, false);  // the autotuner may have changed it
  return QSW_OK;
}

qsw_status_t qsw_superop_copy_csr(qsw_superop_t h, int64_t *row_ptr, int32_t *col, double *val) {
  if (!h) return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  if (row_ptr)
    HIP_TRY(hipMemcpy(row_ptr, h->row_ptr, ((size_t)h->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (col) HIP_TRY(hipMemcpy(col, h->col, (size_t)h->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (val) HIP_TRY(hipMemcpy(val, h->val, (size_t)h->nnz * sizeof(double2), hipMemcpyDeviceToHost));
  return QSW_OK;
}

size_t qsw_propagate_workspace_bytes(qsw_superop_t h, double t0, double dt, int32_t n_steps) {
  if (!h) return 0;
  Plan P;
  if (make_plan(h, t0, dt, n_steps, P) != QSW_OK) return 0;
  return P.total;
}

}  // extern "C"

namespace {

// qsw_propagate on a workspace of ws_bytes (plan P already made).
qsw_status_t propagate_on(qsw_superop_t h, const Plan &P, const void *rho0, double t0, double dt,
                          int32_t n_steps, void *out, void *workspace, size_t ws_bytes,
                          void *hip_stream) {
  if (ws_bytes < P.total || ((uintptr_t)workspace & 255)) return QSW_ERR_STATE;
  const size_t vbytes = (size_t)h->n * sizeof(double2);
  const char *o = (const char *)out;
  const char *r0 = (const char *)rho0;
  if (r0 < o + vbytes * ((size_t)n_steps + 1) && o < r0 + vbytes) return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  char *ws = (char *)workspace;
  const size_t vec = align256(vbytes);
  Runner R;
  R.h = h;
  R.s = s;
  R.st = (DeviceState *)(ws + P.off_state);
  R.B[0] = (double2 *)(ws + P.off_B);
  R.B[1] = (double2 *)(ws + P.off_B + vec);
  R.F[0] = (double2 *)(ws + P.off_F);
  R.F[1] = (double2 *)(ws + P.off_F + vec);
  R.tol = tol_of(h->prec);
  R.engine = launch_engine(h, h->prec != QSW_PREC_DOUBLE);
  const bool fp32 = h->prec == QSW_PREC_FP32;
  if (fp32) {
    // single-precision products: the XCD-banded traversal runs staged
    if (R.engine >= 200) R.engine -= 100;
    const size_t v32 = align256((size_t)h->n * sizeof(float2));
    R.B32[0] = (float2 *)(ws + P.off_B);
    R.B32[1] = (float2 *)(ws + P.off_B + v32);
    for (int c = 0; c < 2; ++c) {
      R.Fh[c] = (float2 *)(ws + P.off_F + (size_t)(2 * c) * v32);
      R.Fl[c] = (float2 *)(ws + P.off_F + (size_t)(2 * c + 1) * v32);
    }
  }
  std::unique_lock<std::mutex> pace_lock;
  if (h->pace > 0 && h->pace_dev) {
    pace_lock = std::unique_lock<std::mutex>(*h->pace_mu);
    R.pace_dev = h->pace_dev;
    R.pace_host = h->pace_host;
    R.seq = &h->pace_seq;
    R.pace = h->pace;
    R.retired = h->pace_seq;
  }
  double2 *outv = (double2 *)out;
  const int64_t n = h->n;
  auto slot = [&](int64_t k) { return outv + k * n; };
  HIP_TRY(hipEventRecord(h->ev_start, s));
  HIP_TRY(launch_zero(R.st, sizeof(DeviceState), s));
  bool fused = false;  // series blocks run through the fused term kernel
  if (fp32) {
    // the state as hi + lo, its trace the reference of every point's check
    HIP_TRY(launch_split_c64((const double2 *)rho0, R.Fh[0], R.Fl[0], n, s));
    HIP_TRY(launch_trace32(R.st, R.Fh[0], R.Fl[0], h->N, 1, s));
    auto emit = [&](int64_t k) -> hipError_t {
      hipError_t e = launch_trace32(R.st, R.Fh[R.cur], R.Fl[R.cur], h->N, 0, s);
      if (e != hipSuccess) return e;
      return launch_emit32(R.st, R.Fh[R.cur], R.Fl[R.cur], slot(k), n, s);
    };
    if (t0 != 0.0) {
      HIP_TRY(R.alg32_f32(t0, P.m0, P.s0));
      HIP_TRY(emit(0));
    } else {
      HIP_TRY(launch_copy(slot(0), (const double2 *)rho0, n, s));
    }
    for (int32_t k = 0; k < n_steps; ++k) {
      HIP_TRY(R.alg32_f32(dt, P.m, P.s));
      HIP_TRY(emit(k + 1));
    }
  } else if (t0 != 0.0)
    HIP_TRY(R.alg32((const double2 *)rho0, slot(0), t0, P.m0, P.s0));
  else
    HIP_TRY(launch_copy(slot(0), (const double2 *)rho0, n, s));
  if (fp32) {
    // done above
  } else if (n_steps > 0 && P.branch == 0) {
    for (int32_t k = 0; k < n_steps; ++k) HIP_TRY(R.alg32(slot(k), slot(k + 1), dt, P.m, P.s));
  } else if (n_steps > 0 && P.d == 1 && env_int("QSW_FUSE_SERIES", 1) != 0) {
    // Time-series blocks of one grid point: the block's powers K_p =
    // (dt/p) L K_{p-1} summed into F = Z + sum K_p with the two-term test on
    // ||K_{p-1}|| + ||K_p|| <= tol ||F|| are the single-time algorithm with
    // (m, 1) on each interval: the same products, sums, tests and order, in
    // the fused term kernel (no separate accumulation pass).
    for (int32_t k = 0; k < n_steps; ++k) HIP_TRY(R.alg32(slot(k), slot(k + 1), dt, P.m, 1));
    fused = true;
  } else if (n_steps > 0) {
    // time-series blocks: K_0 = Z (block start), K_p in the workspace
    PointSlots *pts = (PointSlots *)(ws + P.off_pts);
    std::vector<double2 *> Kp(P.m + 1);
    for (int p = 1; p <= P.m; ++p) Kp[p] = (double2 *)(ws + P.off_K + (size_t)(p - 1) * vec);
    int64_t zi = 0;
    for (int i = 1; i <= P.j + 1; ++i) {
      const int dd = (i <= P.j) ? P.d : P.r;
      if (dd == 0) break;
      const double2 *Z = slot(zi);
      Kp[0] = (double2 *)Z;
      HIP_TRY(launch_series_init(R.st, pts, dd, Z, n, 1024, s));
      for (int k = 1; k <= dd; ++k) {
        double2 *Fk = slot(zi + k);
        PointSlots *pt = pts + (k - 1);
        for (int p = 1; p <= P.m; ++p) {
          SpmvArgs a = R.base_args();
          a.x = Kp[p - 1];
          a.y = Kp[p];
          a.alpha = dt / (double)p;
          HIP_TRY(launch_series_power(a, pt, k, p, R.engine, h->grid, s));
          HIP_TRY(launch_series_accum(R.st, pt, k, p, Kp[p], Z, Fk, n, R.tol, 2048, s));
          R.launched += 1;
        }
      }
      zi += dd;
    }
  }
  HIP_TRY(hipMemcpyAsync(h->stats_dev, &R.st->products, sizeof(unsigned long long),
                         hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->stats_dev + 1, &R.st->nonfinite, sizeof(int), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->stats_dev + 2, &R.st->trace_dev, sizeof(unsigned long long),
                         hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipEventRecord(h->ev_end, s));
  h->last = qsw_stats_t{};
  h->last.branch = P.branch;
  h->last.m = P.m;
  h->last.s = P.s;
  h->last.m0 = P.m0;
  h->last.s0 = P.s0;
  h->last.launched = R.launched;
  h->last.prec = h->prec;
  h->last_fused = fused;
  h->have_last = true;
  return QSW_OK;
}

// Scratch of qsw_propagate_noalloc: one copy per device, held by the device
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address comes from hipGetSymbolAddress, once
// per device (scratch_address), and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[QSW_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of this device's scratch, looked up on the first call on
// the device (which must be current).
hipError_t scratch_address(int dev, void **out) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || ((uintptr_t)ptr & 255)) return hipErrorInvalidSymbol;
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

qsw_status_t qsw_propagate(qsw_superop_t h, const void *rho0, double t0, double dt,
                           int32_t n_steps, void *out, void *workspace, size_t ws_bytes,
                           void *hip_stream) {
  if (!h || !rho0 || !out || !workspace) return QSW_ERR_ARG;
  Plan P;
  qsw_status_t st = make_plan(h, t0, dt, n_steps, P);
  if (st != QSW_OK) return st;
  return propagate_on(h, P, rho0, t0, dt, n_steps, out, workspace, ws_bytes, hip_stream);
}

qsw_status_t qsw_propagate_noalloc(qsw_superop_t h, const void *rho0, double t0, double dt,
                                   int32_t n_steps, void *out, void *hip_stream) {
  if (!h || !rho0 || !out) return QSW_ERR_ARG;
  Plan P;
  qsw_status_t st = make_plan(h, t0, dt, n_steps, P);
  if (st != QSW_OK) return st;
  if (P.total > (size_t)QSW_NOALLOC_SCRATCH_BYTES) return QSW_ERR_SCRATCH;
  void *ws = nullptr;
  {
    DeviceGuard g(h->device);
    if (!g.ok) return QSW_ERR_DEVICE;
    HIP_TRY(scratch_address(h->device, &ws));
  }
  return propagate_on(h, P, rho0, t0, dt, n_steps, out, ws, QSW_NOALLOC_SCRATCH_BYTES,
                      hip_stream);
}

qsw_status_t qsw_last_stats(qsw_superop_t h, qsw_stats_t *st) {
  if (!h || !st) return QSW_ERR_ARG;
  if (!h->have_last) return QSW_ERR_STATE;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  HIP_TRY(hipEventSynchronize(h->ev_end));
  unsigned long long buf[3] = {0, 0, 0};
  HIP_TRY(hipMemcpy(buf, h->stats_dev, sizeof(buf), hipMemcpyDeviceToHost));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev_start, h->ev_end));
  h->last.products = (int64_t)buf[0];
  h->last.nonfinite = (int)(buf[1] & 0xffffffffu) != 0;
  h->last.ms = ms;
  const bool fp32 = h->last.prec == QSW_PREC_FP32;
  double tdev = 0.0;
  std::memcpy(&tdev, &buf[2], sizeof(double));
  h->last.trace_dev = fp32 ? tdev : 0.0;
  const bool single = h->last.prec != QSW_PREC_DOUBLE;
  const bool split = h->split && is_wave_engine(h->engine);
  const double entry = split ? (single ? 8.0 : 12.0) : (single ? 12.0 : 20.0);
  const double diag = split ? (single ? 8.0 : 16.0) : 0.0;
  // the stored-power series adds a separate accumulation pass; single-precision
  // products move x, the term and the hi + lo accumulator in complex64
  const double vec = fp32 ? 48.0 : (h->last.branch == 1 && !h->last_fused ? 80.0 : 64.0);
  const double entries = is_wave_engine(h->engine) ? (double)h->wentries : (double)h->nnz;
  const double shared = is_wave_engine(h->engine) ? 16.0 * (double)h->wshared : 0.0;
  h->last.bytes = (double)h->last.products * (entry * entries + shared + 8.0 * (double)(h->n + 1) +
                                              (diag + vec) * (double)h->n);
  *st = h->last;
  return h->last.nonfinite ? QSW_ERR_NONFINITE : QSW_OK;
}

qsw_status_t qsw_apply(qsw_superop_t h, const void *x, void *y, void *hip_stream) {
  if (!h || !x || !y || x == y) return QSW_ERR_ARG;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  SpmvArgs a{};
  a.n = h->n;
  a.rp = h->row_ptr;
  a.col = h->col;
  a.val = h->val;
  a.x = (const double2 *)x;
  a.y = (double2 *)y;
  a.alpha = 1.0;
  a.rows_per_block = h->rows_per_block;
  a.blk = h->blk;
  a.nblk = h->nblk;
  a.blocks_per_wg = h->blocks_per_wg;
  set_wave(a, h);
  HIP_TRY(launch_spmv(a, launch_engine(h, false), h->grid, (hipStream_t)hip_stream));
  return QSW_OK;
}

qsw_status_t qsw_populations(qsw_superop_t h, const void *rho, int32_t count, void *pops,
                             void *hip_stream) {
  if (!h || !rho || !pops || count < 0) return QSW_ERR_ARG;
  if (count == 0) return QSW_OK;
  DeviceGuard g(h->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  HIP_TRY(launch_populations((const double2 *)rho, h->N, count, (double *)pops,
                             (hipStream_t)hip_stream));
  return QSW_OK;
}

}  // extern "C"
