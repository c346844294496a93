// Proxy-compressed fast direct solver of the mixed Burton-Miller system (Sec. 4.2):
// weak admissibility over a binary tree of boundary cells, the proxy method of
// Fig. (proxy) with the column-pivoted QR targets of Table (tb:low-rank), the
// factorisation A_ij ~ L_i S_ij R_j of eq. (aij=usv) and the compressed system of
// eq. (compressed), applied level by level (recursive skeletonisation) up to a
// dense root.  The leaf blocks use Theorem (thm:LU): U33 = -[M31 M32][M13; M23],
// A_ii^{-1} L_i by Corollary (lem:block_LU) and A_ii^{-1} f_i by Corollary
// (lem:for_ssm_RHS).  Quadrature: the one-point zeta-corrected trapezoid rule, whose
// entries between distinct nodes are point interactions (kernel times trapezoid
// weight), so every off-diagonal block is compressible by the proxy argument.
//
// Host code here keeps the tree and the index lists (which nodes are skeletons, which
// lie inside a proxy circle); every arithmetic step runs in the library's kernels:
// the entry and proxy-target kernel (bm_assemble.hip), the batched column-pivoted QR,
// the Gauss-Jordan inverses and the gathers (bm_fds_kernels.hip), the batched and
// plain MFMA GEMMs (bm_zgemm.hip) and, for blocks above BM_FDS_GJ_MAX, the blocked
// LU with its triangular solves built from GEMMs (bm_getrf.hip).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <map>
#include <new>
#include <vector>

#include "bm_fds.h"

#define BM_FDS_GJ_MAX 1024     // explicit inverses up to this order by Gauss-Jordan
#define BM_FDS_LEAF_MAX 320    // leaf cells of at most this many nodes
#define BM_FDS_BACKSUB_MAX 128 // interpolation solves up to this rank per thread
#define BM_FDS_RCHUNK 32       // right-hand sides per solve pass

namespace {

struct fds_cell {
  int level = 0, index = 0, node0 = 0, nn = 0;
  std::vector<int> rows, cols;  // codes, in the order of the cell's block rows / columns
  double cx = 0, cy = 0, rho = 0, bx0 = 0, by0 = 0, bx1 = 0, by1 = 0;
  int np = 0;
  int k[3] = {0, 0, 0};
  int ktot = 0;
  std::vector<int> rskel, cskel;  // codes, type-major
  int m = 0;                      // order of the cell's diagonal block
  cplx *Abar = nullptr;  // m x m (leaf: 3n x 3n)
  cplx *Ainv = nullptr;  // upper: m x m inverse; leaf: n x n inverse of U33
  cplx *L = nullptr, *R = nullptr, *W = nullptr, *Lam = nullptr;
  // solve buffers (BM_FDS_RCHUNK columns)
  cplx *fb = nullptr, *z = nullptr, *xb = nullptr, *t = nullptr;
  int *gidx = nullptr;  // leaf: global row of each cell unknown
};

bool coupled(int tr, int tc) { return (tr == 0 && tc == 2) || (tr == 1 && tc == 2) || (tr == 2 && tc < 2); }

}  // namespace

struct bm_fds {
  int n = 0, leaf = 0, levels = 0, n_proxy = 0;
  double tol = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  bm_problem shell;
  double *geo = nullptr, *wts = nullptr;
  std::vector<double> hx, hdx;
  std::vector<std::vector<fds_cell>> lv;  // lv[l]: cells of level l (0 = root)
  std::vector<std::pair<void *, size_t>> mem;  // device allocations of the factorisation (address, bytes)
  // idle device buffers by size: (address, generation: the factorisation that last used it)
  std::multimap<size_t, std::pair<void *, long>> spare;
  long gen = 0;  // factorisations started
  std::vector<void *> mem_fixed;
  size_t bytes = 0, bytes_fixed = 0;
  bool factored = false;
  double kmax = 0;
  int32_t *dev_err = nullptr;
  // per-level statistics
  std::vector<int> rank_sum, rank_max;
  int root_n = 0;
  int root_max = 4096;       // order up to which a level's compressed system is the root
  int top = 1;               // the level whose cells make up the root
  std::vector<long> root_off;  // offset of each top-level cell's skeletons in the root
  // a root above the Gauss-Jordan limit: its LU in place of its block, kept for the
  // solve (two triangular solves per pass instead of the product with an inverse)
  bool root_lu = false;
  bm_getrf_ws *root_ws = nullptr;
  int root_ws_n = 0;
  int32_t *root_ipiv = nullptr, *root_perm = nullptr;
  cplx *root_dinv = nullptr;
  // scratch reused by the solve
  std::vector<bm_gemm_desc> hg;
  bm_gemm_desc *dg = nullptr;
  size_t dg_cap = 0;
  std::vector<bm_copy_desc> hc;
  bm_copy_desc *dc = nullptr;
  size_t dc_cap = 0;
};

namespace {

// BM_FDS_VERBOSE=1 in the environment: one line per level and per failing step on stderr
bool verbose() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("BM_FDS_VERBOSE");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}
#define FDS_FAIL(rc, what)                                                      \
  do {                                                                          \
    if (verbose()) fprintf(stderr, "[bm_fds] %s failed: %d\n", what, (int)(rc)); \
  } while (0)

// Device buffers are not freed between factorisations: a factorisation's
// allocations, and the temporary buffers of its steps, become spares that later
// requests of the same size take again (a repeated factorisation of one configuration
// asks for the same sizes).  At the end of a factorisation the spares it found and did
// not take are freed; its own temporaries stay for the next one.  hipFree and
// hipMalloc of gigabytes each cost tens of milliseconds and wait for the device.
// A buffer becomes a spare only once the stream that used it has been synchronised.
void *spare_take(bm_fds *f, size_t bytes) {
  auto it = f->spare.find(bytes);
  if (it == f->spare.end()) return nullptr;
  void *p = it->second.first;
  f->spare.erase(it);
  return p;
}

template <typename T>
int dmalloc(bm_fds *f, T **p, size_t count, bool fixed = false) {
  *p = nullptr;
  if (count == 0) return BM_OK;
  const size_t bytes = sizeof(T) * count;
  if (fixed) {
    if (hipMalloc((void **)p, bytes) != hipSuccess) return BM_E_NOMEM;
    f->mem_fixed.push_back(*p);
    f->bytes_fixed += bytes;
  } else {
    *p = (T *)spare_take(f, bytes);
    if (!*p && hipMalloc((void **)p, bytes) != hipSuccess) return BM_E_NOMEM;
    f->mem.push_back({(void *)*p, bytes});
  }
  f->bytes += bytes;
  return BM_OK;
}

// Temporary buffers of a factorisation step: tmp_get (a spare, else hipMalloc),
// tmp_put_all after the step's stream has been synchronised.
struct tmp_list {
  std::vector<std::pair<void *, size_t>> v;
};
bool tmp_get(bm_fds *f, tmp_list &t, void **p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  *p = spare_take(f, bytes);
  if (!*p && hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  t.v.push_back({*p, bytes});
  return true;
}
void tmp_put_all(bm_fds *f, tmp_list &t) {
  for (const auto &m : t.v) f->spare.emplace(m.second, std::make_pair(m.first, f->gen));
  t.v.clear();
}

// The factorisation's allocations become spares (the caller has synchronised the
// stream that used them).
void free_factor_memory(bm_fds *f) {
  for (const auto &m : f->mem) f->spare.emplace(m.second, std::make_pair(m.first, f->gen));
  f->mem.clear();
  f->lv.clear();
  f->factored = false;
  f->bytes = f->bytes_fixed;
}

// Frees the spares last used before generation g (all: g = LONG_MAX).
void release_spare(bm_fds *f, long g) {
  for (auto it = f->spare.begin(); it != f->spare.end();) {
    if (it->second.second < g) {
      (void)hipFree(it->second.first);
      it = f->spare.erase(it);
    } else {
      ++it;
    }
  }
}

// Upload a host vector to a fresh device buffer (synchronous copy; setup path).
template <typename T>
int upload(bm_fds *f, const std::vector<T> &h, T **d) {
  if (int rc = dmalloc(f, d, h.size())) return rc;
  if (!h.empty()) BM_HIP_TRY(hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return BM_OK;
}

int run_gemms(bm_fds *f, const std::vector<bm_gemm_desc> &g) {
  if (g.empty()) return BM_OK;
  if (g.size() > f->dg_cap) {
    if (f->dg) (void)hipFree(f->dg);
    f->dg_cap = std::max(g.size(), (size_t)1024);
    if (hipMalloc(&f->dg, sizeof(bm_gemm_desc) * f->dg_cap) != hipSuccess) {
      f->dg = nullptr;
      f->dg_cap = 0;
      return BM_E_NOMEM;
    }
  }
  // the descriptors must stay valid until the copy has executed: synchronise after it
  BM_HIP_TRY(hipMemcpyAsync(f->dg, g.data(), sizeof(bm_gemm_desc) * g.size(), hipMemcpyHostToDevice, f->stream));
  int max_tiles = 0;
  for (const auto &d : g) max_tiles = std::max(max_tiles, ((d.m + 63) / 64) * ((d.n + 63) / 64));
  int rc = bm_launch_zgemm_batched(f->stream, (int)g.size(), f->dg, max_tiles);
  BM_HIP_TRY(hipStreamSynchronize(f->stream));
  return rc;
}

int run_copies(bm_fds *f, const std::vector<bm_copy_desc> &c) {
  if (c.empty()) return BM_OK;
  if (c.size() > f->dc_cap) {
    if (f->dc) (void)hipFree(f->dc);
    f->dc_cap = std::max(c.size(), (size_t)1024);
    if (hipMalloc(&f->dc, sizeof(bm_copy_desc) * f->dc_cap) != hipSuccess) {
      f->dc = nullptr;
      f->dc_cap = 0;
      return BM_E_NOMEM;
    }
  }
  BM_HIP_TRY(hipMemcpyAsync(f->dc, c.data(), sizeof(bm_copy_desc) * c.size(), hipMemcpyHostToDevice, f->stream));
  int rc = bm_fds_copy_blocks(f->stream, (int)c.size(), f->dc);
  BM_HIP_TRY(hipStreamSynchronize(f->stream));
  return rc;
}

bm_gemm_desc gemm(int m, int n, int k, cplx alpha, const cplx *A, long lda, const cplx *B, long ldb, cplx beta, cplx *C,
                  long ldc) {
  bm_gemm_desc d;
  d.m = m;
  d.n = n;
  d.k = k;
  d.alpha = alpha;
  d.beta = beta;
  d.A = A;
  d.lda = lda;
  d.B = B;
  d.ldb = ldb;
  d.C = C;
  d.ldc = ldc;
  return d;
}

bm_copy_desc copyd(const cplx *A, long lda, cplx *B, long ldb, int m, int n) {
  bm_copy_desc d;
  d.A = A;
  d.lda = lda;
  d.B = B;
  d.ldb = ldb;
  d.m = m;
  d.n = n;
  return d;
}

const cplx ONE = {1.0, 0.0}, MONE = {-1.0, 0.0}, ZERO = {0.0, 0.0};

// ---------------------------------------------------------------------------
// Blocked triangular solves with the factors of bm_getrf_run (packed L\U, ld) and the
// inverses of their 64 x 64 diagonal blocks (dinv): X (n x nc, ldx) <- L^{-1} X or
// U^{-1} X, each block a product with the block's inverse and a GEMM update of the
// rows below (above).  T: 64 x nc scratch.
// ---------------------------------------------------------------------------
int blocked_trsm(hipStream_t s, bool lower, int n, const cplx *LU, long ld, const cplx *dinv, cplx *X, long ldx,
                 int nc, cplx *T) {
  const int nb = (n + 63) / 64;
  for (int q = 0; q < nb; ++q) {
    const int b = lower ? q : nb - 1 - q;
    const int r0 = 64 * b, nbr = std::min(64, n - r0);
    const cplx *Dv = dinv + (size_t)b * BM_DINV_TILES * 4096 + (lower ? 0 : 4096);
    if (int rc = bm_launch_zgemm(s, nbr, nc, nbr, ONE, Dv, 64, X + r0, ldx, ZERO, T, 64)) return rc;
    BM_HIP_TRY(hipMemcpy2DAsync(X + r0, sizeof(cplx) * ldx, T, sizeof(cplx) * 64, sizeof(cplx) * nbr, nc,
                                hipMemcpyDeviceToDevice, s));
    if (lower && r0 + nbr < n) {
      if (int rc = bm_launch_zgemm(s, n - r0 - nbr, nc, nbr, MONE, LU + (r0 + nbr) + (long)r0 * ld, ld, T, 64, ONE,
                                   X + r0 + nbr, ldx))
        return rc;
    } else if (!lower && r0 > 0) {
      if (int rc = bm_launch_zgemm(s, r0, nc, nbr, MONE, LU + (long)r0 * ld, ld, T, 64, ONE, X, ldx)) return rc;
    }
  }
  return BM_OK;
}

// Explicit inverses of square blocks: Gauss-Jordan in one launch for the small ones,
// the blocked LU and triangular solves with the identity for the others.  The input
// blocks are overwritten.
struct inv_job {
  cplx *A;  // n x n, ld n (overwritten)
  cplx *Ainv;  // n x n, ld n (may equal A only for the small path)
  int n;
};

#define BM_FDS_GJ_REFINE_MIN 321  // Gauss-Jordan inverses of this order and above get a Newton-Schulz step

int refine_inverses(bm_fds *f, const std::vector<inv_job> &jobs) {
  std::vector<bm_copy_desc> cp;
  std::vector<bm_gemm_desc> g1, g2;
  tmp_list tl;
  for (const auto &j : jobs) {
    if (j.n < BM_FDS_GJ_REFINE_MIN || j.n > BM_FDS_GJ_MAX || j.Ainv == j.A) continue;
    cplx *X0 = nullptr, *T = nullptr;
    const size_t nn = (size_t)j.n * j.n;
    if (!tmp_get(f, tl, (void **)&X0, sizeof(cplx) * nn) || !tmp_get(f, tl, (void **)&T, sizeof(cplx) * nn)) {
      (void)hipStreamSynchronize(f->stream);
      tmp_put_all(f, tl);
      return BM_E_NOMEM;
    }
    cp.push_back(copyd(j.Ainv, j.n, X0, j.n, j.n, j.n));
    g1.push_back(gemm(j.n, j.n, j.n, ONE, j.A, j.n, X0, j.n, ZERO, T, j.n));
    g2.push_back(gemm(j.n, j.n, j.n, MONE, X0, j.n, T, j.n, cmk(2.0, 0.0), j.Ainv, j.n));
  }
  int rc = BM_OK;
  if (!cp.empty()) {
    rc = run_copies(f, cp);
    if (!rc) rc = run_gemms(f, g1);
    if (!rc) rc = run_gemms(f, g2);
  }
  (void)hipStreamSynchronize(f->stream);
  tmp_put_all(f, tl);
  return rc;
}

int invert(bm_fds *f, const std::vector<inv_job> &jobs) {
  hipStream_t s = f->stream;
  std::vector<bm_inv_desc> small;
  std::vector<bm_copy_desc> cp;
  int nmax_small = 0, nmax_big = 0;
  for (const auto &j : jobs) {
    if (j.n <= 0) continue;
    if (j.n <= BM_FDS_GJ_MAX) {
      if (j.Ainv != j.A) cp.push_back(copyd(j.A, j.n, j.Ainv, j.n, j.n, j.n));
      bm_inv_desc d;
      d.A = j.Ainv;
      d.ld = j.n;
      d.n = j.n;
      small.push_back(d);
      nmax_small = std::max(nmax_small, j.n);
    } else {
      nmax_big = std::max(nmax_big, j.n);
    }
  }
  if (int rc = run_copies(f, cp)) return rc;
  if (!small.empty()) {
    bm_inv_desc *dd = nullptr;
    int *info = nullptr, *pivw = nullptr;
    tmp_list tl;
    bool ok = tmp_get(f, tl, (void **)&dd, sizeof(bm_inv_desc) * small.size()) &&
              tmp_get(f, tl, (void **)&info, sizeof(int) * small.size()) &&
              tmp_get(f, tl, (void **)&pivw, sizeof(int) * small.size() * nmax_small);
    int rc = ok ? BM_OK : BM_E_NOMEM;
    if (ok && hipMemcpy(dd, small.data(), sizeof(bm_inv_desc) * small.size(), hipMemcpyHostToDevice) != hipSuccess)
      rc = BM_E_HIP;
    if (!rc) rc = bm_fds_gj_inverse(s, (int)small.size(), dd, nmax_small, info, pivw);
    std::vector<int> hi(small.size(), 0);
    if (!rc && (hipStreamSynchronize(s) != hipSuccess ||
                hipMemcpy(hi.data(), info, sizeof(int) * small.size(), hipMemcpyDeviceToHost) != hipSuccess))
      rc = BM_E_HIP;
    (void)hipStreamSynchronize(s);
    tmp_put_all(f, tl);
    if (rc) return rc;
    for (size_t q = 0; q < hi.size(); ++q)
      if (hi[q]) {
        if (verbose()) fprintf(stderr, "[bm_fds] Gauss-Jordan: block %zu of order %d has a zero pivot at %d\n", q,
                               small[q].n, hi[q]);
        return BM_E_DEVICE;  // an exactly singular block
      }
    // Gauss-Jordan loses accuracy on the larger, worse-conditioned blocks of the
    // upper levels: there one Newton-Schulz step X <- 2X - X A X (the error of X
    // squared) with the original block, T = A X0 and X = -X0 T + 2 X, X0 a copy of X
    if (int rc2 = refine_inverses(f, jobs)) return rc2;
  }
  if (nmax_big > 0) {
    bm_getrf_ws *w = bm_getrf_ws_create(nmax_big);
    int32_t *ipiv = nullptr, *perm = nullptr;
    cplx *dinv = nullptr, *T = nullptr;
    const int nblk = (nmax_big + 63) / 64;
    tmp_list tl;
    bool ok = w && tmp_get(f, tl, (void **)&ipiv, sizeof(int32_t) * nmax_big) &&
              tmp_get(f, tl, (void **)&perm, sizeof(int32_t) * nmax_big) &&
              tmp_get(f, tl, (void **)&dinv, sizeof(cplx) * (size_t)nblk * BM_DINV_TILES * 4096) &&
              tmp_get(f, tl, (void **)&T, sizeof(cplx) * 64 * (size_t)nmax_big);
    int rc = ok ? BM_OK : BM_E_NOMEM;
    for (const auto &j : jobs) {
      if (rc || j.n <= BM_FDS_GJ_MAX) continue;
      rc = bm_getrf_run(s, j.n, j.A, j.n, ipiv, f->dev_err, w, 0);
      if (!rc) rc = bm_launch_diag_inverses(s, j.n, j.A, j.n, dinv);
      if (!rc) rc = bm_launch_perm(s, w, j.n, perm);
      if (!rc) rc = bm_fds_perm_identity(s, j.n, perm, j.Ainv, j.n);
      if (!rc) rc = blocked_trsm(s, true, j.n, j.A, j.n, dinv, j.Ainv, j.n, j.n, T);
      if (!rc) rc = blocked_trsm(s, false, j.n, j.A, j.n, dinv, j.Ainv, j.n, j.n, T);
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = BM_E_HIP;
    bm_getrf_ws_destroy(w);
    (void)hipStreamSynchronize(s);
    tmp_put_all(f, tl);
    if (rc) return rc;
    int32_t h[2] = {0, 0};
    BM_HIP_TRY(hipMemcpy(h, f->dev_err, sizeof(h), hipMemcpyDeviceToHost));
    if (h[0] || h[1]) {
      if (verbose()) fprintf(stderr, "[bm_fds] blocked LU: error flag %d, zero pivot %d\n", h[0], h[1]);
      return BM_E_DEVICE;  // a bounded wait expired, or an exactly singular block
    }
  }
  return BM_OK;
}

// Entries of the explicit matrix (mode 0 targets) into dense blocks at base + off.
struct entry_job {
  const std::vector<int> *rows, *cols;
  long off;
  int ld;
};

int entries(bm_fds *f, cplx *base, const std::vector<entry_job> &jobs) {
  if (jobs.empty()) return BM_OK;
  std::vector<int> codes;
  std::vector<long> roff, coff;
  for (const auto &j : jobs) {
    roff.push_back((long)codes.size());
    codes.insert(codes.end(), j.rows->begin(), j.rows->end());
    coff.push_back((long)codes.size());
    codes.insert(codes.end(), j.cols->begin(), j.cols->end());
  }
  int *dcodes = nullptr;
  fds_tgt *ditems = nullptr;
  int rc = BM_OK;
  tmp_list tl;
  if (!tmp_get(f, tl, (void **)&dcodes, sizeof(int) * std::max<size_t>(codes.size(), 1)) ||
      !tmp_get(f, tl, (void **)&ditems, sizeof(fds_tgt) * jobs.size()))
    rc = BM_E_NOMEM;
  std::vector<fds_tgt> items;
  long maxe = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    fds_tgt t;
    memset(&t, 0, sizeof(t));
    t.M = (int)jobs[q].rows->size();
    t.C = (int)jobs[q].cols->size();
    t.ld = jobs[q].ld;
    t.mode = 0;
    t.off = jobs[q].off;
    t.rl = dcodes + roff[q];
    t.cl = dcodes + coff[q];
    items.push_back(t);
    maxe = std::max(maxe, (long)t.M * t.C);
  }
  if (!rc && !codes.empty() && hipMemcpy(dcodes, codes.data(), sizeof(int) * codes.size(), hipMemcpyHostToDevice) != hipSuccess)
    rc = BM_E_HIP;
  if (!rc && hipMemcpy(ditems, items.data(), sizeof(fds_tgt) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
    rc = BM_E_HIP;
  if (!rc) rc = bm_launch_fds_targets(f->stream, &f->shell, (int)items.size(), ditems, maxe, base);
  if (hipStreamSynchronize(f->stream) != hipSuccess && !rc) rc = BM_E_HIP;
  tmp_put_all(f, tl);
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Factorisation
// ---------------------------------------------------------------------------
namespace {

// Per-level stacked storage: cell i's rows start at off[i] of a matrix with ld rows.
struct stacked {
  std::vector<long> off;
  long ld = 0;
};

void cell_geometry(bm_fds *f, fds_cell &c) {
  double x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300;
  for (int v = c.node0; v < c.node0 + c.nn; ++v) {
    const double x = f->hx[2 * v], y = f->hx[2 * v + 1];
    x0 = std::min(x0, x);
    x1 = std::max(x1, x);
    y0 = std::min(y0, y);
    y1 = std::max(y1, y);
  }
  c.bx0 = x0;
  c.by0 = y0;
  c.bx1 = x1;
  c.by1 = y1;
  c.cx = 0.5 * (x0 + x1);
  c.cy = 0.5 * (y0 + y1);
  c.rho = 0.75 * hypot(x1 - x0, y1 - y0);
  const int want = (int)ceil((2.0 * f->kmax * c.rho + 64.0) / 8.0) * 8;
  c.np = std::max(f->n_proxy, want);
}

bool inside(const bm_fds *f, const fds_cell &c, int code) {
  const int v = FDS_CODE_NODE(code);
  const double dx = f->hx[2 * v] - c.cx, dy = f->hx[2 * v + 1] - c.cy;
  return dx * dx + dy * dy < c.rho * c.rho;
}

bool box_near(const fds_cell &c, const fds_cell &o) {
  const double dx = std::max(std::max(o.bx0 - c.cx, 0.0), c.cx - o.bx1);
  const double dy = std::max(std::max(o.by0 - c.cy, 0.0), c.cy - o.by1);
  return dx * dx + dy * dy < c.rho * c.rho;
}

struct qr_host {
  int cell, type, side;  // side 0: column skeleton (R), 1: row skeleton (L)
  std::vector<int> near, cand, pos;
  int M = 0, C = 0;
};

// Column-pivoted QR of every target of a level, skeletons and interpolation matrices
// written into the cells' L and R (allocated here, zero outside the type blocks).
int compress_level(bm_fds *f, std::vector<fds_cell> &cells) {
  hipStream_t s = f->stream;
  const int nc = (int)cells.size();
  std::vector<qr_host> Q;
  Q.reserve(6 * nc);
  for (int ci = 0; ci < nc; ++ci) {
    fds_cell &c = cells[ci];
    std::vector<const fds_cell *> nb;
    for (int oi = 0; oi < nc; ++oi)
      if (oi != ci && box_near(c, cells[oi])) nb.push_back(&cells[oi]);
    for (int t = 0; t < 3; ++t)
      for (int side = 0; side < 2; ++side) {
        qr_host q;
        q.cell = ci;
        q.type = t;
        q.side = side;
        const std::vector<int> &own = side ? c.rows : c.cols;
        for (int i = 0; i < (int)own.size(); ++i)
          if (FDS_CODE_TYPE(own[i]) == t) {
            q.cand.push_back(own[i]);
            q.pos.push_back(i);
          }
        for (const fds_cell *o : nb) {
          const std::vector<int> &lst = side ? o->cols : o->rows;
          for (int code : lst) {
            const int ot = FDS_CODE_TYPE(code);
            if ((side ? coupled(t, ot) : coupled(ot, t)) && inside(f, c, code)) q.near.push_back(code);
          }
        }
        const int nps = (side && t == 2) ? 2 * c.np : c.np;
        q.M = nps + (int)q.near.size();
        q.C = (int)q.cand.size();
        if (q.M > BM_FDS_QR_MAX_ROWS) return BM_E_ARG;
        Q.push_back(std::move(q));
      }
  }
  const int nprob = (int)Q.size();
  // targets
  std::vector<int> codes;
  std::vector<fds_tgt> items(nprob);
  std::vector<bm_qr_prob> probs(nprob);
  std::vector<long> near_off(nprob), cand_off(nprob), pos_off(nprob);
  long work_elems = 0, ncol = 0, npiv = 0;
  int nwg = 0, max_rows = 0, max_c = 0;
  long max_e = 0;
  for (int b = 0; b < nprob; ++b) {
    const qr_host &q = Q[b];
    near_off[b] = (long)codes.size();
    codes.insert(codes.end(), q.near.begin(), q.near.end());
    cand_off[b] = (long)codes.size();
    codes.insert(codes.end(), q.cand.begin(), q.cand.end());
    pos_off[b] = (long)codes.size();
    codes.insert(codes.end(), q.pos.begin(), q.pos.end());
    bm_qr_prob &P = probs[b];
    memset(&P, 0, sizeof(P));
    P.M = q.M;
    P.C = q.C;
    P.off = work_elems;
    P.noff = ncol;
    P.poff = npiv;
    P.kmin = 0;
    P.kcap = std::min(q.M, q.C);
    P.wg0 = nwg;
    P.wgs = std::max(1, (q.C + BM_FDS_QR_CW - 1) / BM_FDS_QR_CW);
    work_elems += (long)q.M * q.C;
    ncol += q.C;
    npiv += P.kcap;
    nwg += P.wgs;
    max_rows = std::max(max_rows, q.M);
    max_c = std::max(max_c, q.C);
    max_e = std::max(max_e, (long)q.M * q.C);
  }
  // device buffers of the level (freed at the end)
  tmp_list tl;
  auto talloc = [&](void **p, size_t bytes) -> bool { return tmp_get(f, tl, p, bytes); };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    tmp_put_all(f, tl);
  };
  int *dcodes;
  cplx *work;
  fds_tgt *ditems;
  bm_qr_prob *dprobs;
  int *wg2p, *active;
  bm_qr_state st;
  bool ok = talloc((void **)&dcodes, sizeof(int) * codes.size()) && talloc((void **)&work, sizeof(cplx) * work_elems) &&
            talloc((void **)&ditems, sizeof(fds_tgt) * nprob) && talloc((void **)&dprobs, sizeof(bm_qr_prob) * nprob) &&
            talloc((void **)&wg2p, sizeof(int) * nwg) && talloc((void **)&active, sizeof(int)) &&
            talloc((void **)&st.nrm2, sizeof(double) * ncol) && talloc((void **)&st.ex2, sizeof(double) * ncol) &&
            talloc((void **)&st.pivd, sizeof(int) * ncol) && talloc((void **)&st.rest, sizeof(int) * ncol) &&
            talloc((void **)&st.perm, sizeof(int) * npiv) && talloc((void **)&st.alpha, sizeof(cplx) * npiv) &&
            talloc((void **)&st.bestv, sizeof(double) * 2 * nwg) && talloc((void **)&st.bestc, sizeof(int) * 2 * nwg) &&
            talloc((void **)&st.step, sizeof(int) * 2 * nprob) && talloc((void **)&st.done, sizeof(int) * nprob) &&
            talloc((void **)&st.rank, sizeof(int) * nprob) && talloc((void **)&st.r00, sizeof(double) * nprob);
  if (!ok) {
    cleanup();
    return BM_E_NOMEM;
  }
  int rc = BM_OK;
  if (hipMemcpy(dcodes, codes.data(), sizeof(int) * codes.size(), hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  for (int b = 0; b < nprob; ++b) {
    const qr_host &q = Q[b];
    const fds_cell &c = cells[q.cell];
    fds_tgt &t = items[b];
    memset(&t, 0, sizeof(t));
    t.M = q.M;
    t.C = q.C;
    t.ld = q.M;
    t.mode = q.side ? 2 : 1;
    t.ctype = q.type;
    t.np = c.np;
    t.off = probs[b].off;
    t.cx = c.cx;
    t.cy = c.cy;
    t.rho = c.rho;
    t.pw = 2.0 * BM_PI * c.rho / c.np;
    t.rl = dcodes + near_off[b];
    t.cl = dcodes + cand_off[b];
  }
  std::vector<int> hwg(nwg);
  for (int b = 0; b < nprob; ++b)
    for (int w = 0; w < probs[b].wgs; ++w) hwg[probs[b].wg0 + w] = b;
  if (!rc && hipMemcpy(ditems, items.data(), sizeof(fds_tgt) * nprob, hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  if (!rc && hipMemcpy(wg2p, hwg.data(), sizeof(int) * nwg, hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  if (!rc && hipMemcpy(dprobs, probs.data(), sizeof(bm_qr_prob) * nprob, hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  // the targets (Table tb:low-rank), in launches of at most 65535 items
  for (int b0 = 0; b0 < nprob && !rc; b0 += 65535)
    rc = bm_launch_fds_targets(s, &f->shell, std::min(65535, nprob - b0), ditems + b0, max_e, work);
  if (!rc) rc = bm_fds_cpqr_prepare();
  if (!rc) rc = bm_fds_cpqr_init(s, nwg, dprobs, wg2p, work, st);
  int L = 0;
  auto run_steps = [&](int nact) -> int {
    BM_HIP_TRY(hipMemcpy(active, &nact, sizeof(int), hipMemcpyHostToDevice));
    int kcap_max = 0;
    for (const auto &P : probs) kcap_max = std::max(kcap_max, P.kcap);
    for (int it = 0; it <= kcap_max + 8; it += 8) {
      for (int q = 0; q < 8; ++q)
        if (int r = bm_fds_cpqr_step(s, nwg, dprobs, wg2p, work, st, L++, f->tol, active, max_rows)) return r;
      int h = 0;
      BM_HIP_TRY(hipMemcpy(&h, active, sizeof(int), hipMemcpyDeviceToHost));
      if (h <= 0) return BM_OK;
    }
    return BM_E_DEVICE;  // more steps than pivots: cannot happen
  };
  if (!rc) rc = run_steps(nprob);
  std::vector<int> rank(nprob), done(nprob, 1);
  if (!rc && hipMemcpy(rank.data(), st.rank, sizeof(int) * nprob, hipMemcpyDeviceToHost) != hipSuccess) rc = BM_E_HIP;
  // rows and columns of a cell get the same count per type: the larger rank, within
  // what both targets allow; a second pass continues the smaller one
  std::vector<int> kk(nc * 3, 0);
  int resumed = 0;
  if (!rc) {
    for (int ci = 0; ci < nc; ++ci)
      for (int t = 0; t < 3; ++t) {
        const int bc = 6 * ci + 2 * t, br = bc + 1;
        int k = std::max(rank[bc], rank[br]);
        k = std::min(k, std::min(probs[bc].kcap, probs[br].kcap));
        kk[3 * ci + t] = k;
        for (int b : {bc, br})
          if (rank[b] < k) {
            probs[b].kmin = k;
            done[b] = 0;
            ++resumed;
          }
      }
    if (resumed) {
      if (hipMemcpy(dprobs, probs.data(), sizeof(bm_qr_prob) * nprob, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(st.done, done.data(), sizeof(int) * nprob, hipMemcpyHostToDevice) != hipSuccess)
        rc = BM_E_HIP;
      if (!rc) rc = run_steps(resumed);
      if (!rc && hipMemcpy(rank.data(), st.rank, sizeof(int) * nprob, hipMemcpyDeviceToHost) != hipSuccess) rc = BM_E_HIP;
    }
  }
  // final counts (a target whose columns ran out lowers both sides to its rank)
  if (!rc) {
    for (int ci = 0; ci < nc; ++ci)
      for (int t = 0; t < 3; ++t) {
        const int bc = 6 * ci + 2 * t, br = bc + 1;
        const int k = std::min(kk[3 * ci + t], std::min(rank[bc], rank[br]));
        kk[3 * ci + t] = k;
        rank[bc] = rank[br] = k;
      }
    if (hipMemcpy(st.rank, rank.data(), sizeof(int) * nprob, hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  }
  // skeletons, in pivot order, type-major
  std::vector<int> hperm(npiv);
  if (!rc && hipMemcpy(hperm.data(), st.perm, sizeof(int) * npiv, hipMemcpyDeviceToHost) != hipSuccess) rc = BM_E_HIP;
  if (!rc) {
    for (int ci = 0; ci < nc; ++ci) {
      fds_cell &c = cells[ci];
      c.rskel.clear();
      c.cskel.clear();
      c.ktot = 0;
      for (int t = 0; t < 3; ++t) {
        const int k = kk[3 * ci + t];
        c.k[t] = k;
        c.ktot += k;
        const int bc = 6 * ci + 2 * t, br = bc + 1;
        for (int j = 0; j < k; ++j) {
          c.cskel.push_back(Q[bc].cand[hperm[probs[bc].poff + j]]);
          c.rskel.push_back(Q[br].cand[hperm[probs[br].poff + j]]);
        }
      }
      // the cell's L (m x k) and R (k x m)
      c.m = (int)c.rows.size();
      if (!rc) rc = dmalloc(f, &c.L, (size_t)c.m * c.ktot);
      if (!rc) rc = dmalloc(f, &c.R, (size_t)c.ktot * c.m);
      if (!rc && c.ktot > 0) {
        if (hipMemsetAsync(c.L, 0, sizeof(cplx) * c.m * c.ktot, s) != hipSuccess ||
            hipMemsetAsync(c.R, 0, sizeof(cplx) * c.ktot * c.m, s) != hipSuccess)
          rc = BM_E_HIP;
      }
    }
  }
  // interpolation matrices: R11^{-1} R12 and the scatter into L and R
  long r11 = 0, r12 = 0;
  for (int b = 0; b < nprob && !rc; ++b) {
    const int ci = Q[b].cell, t = Q[b].type;
    const fds_cell &c = cells[ci];
    bm_qr_prob &P = probs[b];
    const int k = rank[b];
    P.r11off = r11;
    P.r12off = r12;
    r11 += (long)k * k;
    r12 += (long)k * (P.C - k);
    int o0 = 0;
    for (int u = 0; u < t; ++u) o0 += c.k[u];
    P.o0 = o0;
    P.pos = dcodes + pos_off[b];
    if (Q[b].side == 0) {
      P.out = c.R;
      P.ldo = c.ktot;
      P.conj_out = 0;
    } else {
      P.out = c.L;
      P.ldo = c.m;
      P.conj_out = 1;
    }
  }
  cplx *R11 = nullptr, *R12 = nullptr;
  if (!rc && !(talloc((void **)&R11, sizeof(cplx) * r11) && talloc((void **)&R12, sizeof(cplx) * r12))) rc = BM_E_NOMEM;
  if (!rc && hipMemcpy(dprobs, probs.data(), sizeof(bm_qr_prob) * nprob, hipMemcpyHostToDevice) != hipSuccess) rc = BM_E_HIP;
  if (!rc) rc = bm_fds_cpqr_finish(s, nprob, dprobs, work, st, R11, R12, max_c, BM_FDS_BACKSUB_MAX);
  // larger ranks: blocked upper-triangular solve with the inverses of R11's diagonal blocks
  int kbig = 0;
  for (int b = 0; b < nprob; ++b)
    if (rank[b] > BM_FDS_BACKSUB_MAX) kbig = std::max(kbig, rank[b]);
  if (!rc && kbig > 0) rc = bm_getrf_prepare();  // (LDS limit of the diagonal-inverse kernel)
  if (!rc && kbig > 0) {
    cplx *dinv = nullptr, *T = nullptr;
    const int nblk = (kbig + 63) / 64;
    if (!talloc((void **)&dinv, sizeof(cplx) * (size_t)nblk * BM_DINV_TILES * 4096) ||
        !talloc((void **)&T, sizeof(cplx) * 64 * (size_t)std::max(max_c, 1)))
      rc = BM_E_NOMEM;
    for (int b = 0; b < nprob && !rc; ++b) {
      const int k = rank[b];
      if (k <= BM_FDS_BACKSUB_MAX || probs[b].C - k <= 0) continue;
      rc = bm_launch_diag_inverses(s, k, R11 + probs[b].r11off, k, dinv);
      if (!rc)
        rc = blocked_trsm(s, false, k, R11 + probs[b].r11off, k, dinv, R12 + probs[b].r12off, k, probs[b].C - k, T);
    }
  }
  if (!rc) rc = bm_fds_cpqr_scatter(s, nprob, dprobs, st, R12, max_c);
  cleanup();
  return rc;
}

// One leaf's W = A_ii^{-1} L_i by Corollary lem:block_LU with the blocks of A_ii
// (Abar, 3n x 3n: [M13; M23] = Abar[0:2n, 2n:3n], [M31 M32] = Abar[2n:3n, 0:2n]) and
// the inverse of U33 = -[M31 M32][M13; M23] (Ainv, n x n):
//   Y = [M31 M32] L[0:2n, :] - L[2n:3n, :],  Z = -U33^{-1} Y  (= [Z31 Z32 Z33]),
//   W[2n:3n, :] = Z,  W[0:2n, :] = L[0:2n, :] - [M13; M23] Z.
int leaf_solve_block_rhs(bm_fds *f, std::vector<fds_cell> &cells) {
  const int n = f->leaf;
  std::vector<bm_copy_desc> cp;
  std::vector<bm_gemm_desc> g1, g2, g3;
  for (size_t i = 0; i < cells.size(); ++i) {
    fds_cell &c = cells[i];
    if (int rc = dmalloc(f, &c.W, (size_t)3 * n * c.ktot)) return rc;
    if (c.ktot == 0) continue;
    cp.push_back(copyd(c.L, 3 * n, c.W, 3 * n, 3 * n, c.ktot));  // W = L
  }
  if (int rc = run_copies(f, cp)) return rc;
  for (auto &c : cells) {
    if (c.ktot == 0) continue;
    // Y = [M31 M32] L[0:2n, :] - L[2n:3n, :]  (held in W[2n:3n, :])
    g1.push_back(gemm(n, c.ktot, 2 * n, ONE, c.Abar + 2 * n, 3 * n, c.L, 3 * n, MONE, c.W + 2 * n, 3 * n));
  }
  if (int rc = run_gemms(f, g1)) return rc;
  // Z = -U33^{-1} Y: through a scratch block per cell
  std::vector<cplx *> Z(cells.size(), nullptr);
  tmp_list tl;
  for (size_t i = 0; i < cells.size(); ++i) {
    fds_cell &c = cells[i];
    if (c.ktot == 0) continue;
    if (!tmp_get(f, tl, (void **)&Z[i], sizeof(cplx) * (size_t)n * c.ktot)) {
      tmp_put_all(f, tl);  // (nothing has used them yet)
      return BM_E_NOMEM;
    }
    g2.push_back(gemm(n, c.ktot, n, MONE, c.Ainv, n, c.W + 2 * n, 3 * n, ZERO, Z[i], n));
  }
  int rc = run_gemms(f, g2);
  cp.clear();
  for (size_t i = 0; i < cells.size() && !rc; ++i)
    if (cells[i].ktot) cp.push_back(copyd(Z[i], n, cells[i].W + 2 * n, 3 * n, n, cells[i].ktot));
  if (!rc) rc = run_copies(f, cp);
  for (auto &c : cells)
    if (c.ktot) g3.push_back(gemm(2 * n, c.ktot, n, MONE, c.Abar + (long)2 * n * 3 * n, 3 * n, c.W + 2 * n, 3 * n, ONE,
                                  c.W, 3 * n));
  if (!rc) rc = run_gemms(f, g3);
  (void)hipStreamSynchronize(f->stream);
  tmp_put_all(f, tl);
  return rc;
}

// Lambda_i = (R_i W_i)^{-1} for every cell of a level.
int level_lambda(bm_fds *f, std::vector<fds_cell> &cells) {
  std::vector<bm_gemm_desc> g;
  std::vector<inv_job> jobs;
  tmp_list tl;
  for (auto &c : cells) {
    if (int rc = dmalloc(f, &c.Lam, (size_t)c.ktot * c.ktot)) {
      tmp_put_all(f, tl);  // (nothing has used them yet)
      return rc;
    }
    if (c.ktot == 0) continue;
    cplx *RW = nullptr;
    if (!tmp_get(f, tl, (void **)&RW, sizeof(cplx) * (size_t)c.ktot * c.ktot)) {
      tmp_put_all(f, tl);
      return BM_E_NOMEM;
    }
    g.push_back(gemm(c.ktot, c.ktot, c.m, ONE, c.R, c.ktot, c.W, c.m, ZERO, RW, c.ktot));
    inv_job j;
    j.A = RW;
    j.Ainv = c.Lam;
    j.n = c.ktot;
    jobs.push_back(j);
  }
  int rc = run_gemms(f, g);
  if (!rc) rc = invert(f, jobs);
  (void)hipStreamSynchronize(f->stream);
  tmp_put_all(f, tl);
  return rc;
}

// The parents' diagonal blocks [[Lambda_a, S_ab], [S_ba, Lambda_b]] (S: entries of the
// explicit matrix between the children's skeletons).
int assemble_parents(bm_fds *f, std::vector<fds_cell> &kids, std::vector<fds_cell> &par, int level) {
  par.clear();
  par.resize(kids.size() / 2);
  size_t total = 0;
  for (size_t i = 0; i < par.size(); ++i) {
    fds_cell &a = kids[2 * i], &b = kids[2 * i + 1], &P = par[i];
    P.level = level;
    P.index = (int)i;
    P.node0 = a.node0;
    P.nn = a.nn + b.nn;
    P.rows = a.rskel;
    P.rows.insert(P.rows.end(), b.rskel.begin(), b.rskel.end());
    P.cols = a.cskel;
    P.cols.insert(P.cols.end(), b.cskel.begin(), b.cskel.end());
    P.m = (int)P.rows.size();
    total += (size_t)P.m * P.m;
  }
  cplx *arena = nullptr;
  if (int rc = dmalloc(f, &arena, total)) return rc;
  std::vector<bm_copy_desc> cp;
  std::vector<entry_job> ej;
  long off = 0;
  for (size_t i = 0; i < par.size(); ++i) {
    fds_cell &a = kids[2 * i], &b = kids[2 * i + 1], &P = par[i];
    P.Abar = arena + off;
    const int ka = a.ktot, kb = b.ktot, m = P.m;
    if (ka) cp.push_back(copyd(a.Lam, ka, P.Abar, m, ka, ka));
    if (kb) cp.push_back(copyd(b.Lam, kb, P.Abar + ka + (long)ka * m, m, kb, kb));
    if (ka && kb) {
      entry_job e1 = {&a.rskel, &b.cskel, off + (long)ka * m, m};
      entry_job e2 = {&b.rskel, &a.cskel, off + ka, m};
      ej.push_back(e1);
      ej.push_back(e2);
    }
    off += (long)m * m;
  }
  if (int rc = run_copies(f, cp)) return rc;
  return entries(f, arena, ej);
}

// The root: the compressed system of every cell of the top level together, the
// cells' Lambda blocks on the diagonal and the matrix entries between one cell's
// row skeletons and another's column skeletons elsewhere (what assemble_parents
// does for two cells).
int assemble_root(bm_fds *f, std::vector<fds_cell> &kids) {
  std::vector<fds_cell> &top = f->lv[0];
  top.clear();
  top.resize(1);
  fds_cell &P = top[0];
  P.level = 0;
  P.index = 0;
  P.node0 = 0;
  P.nn = f->n;
  f->root_off.assign(kids.size(), 0);
  long o = 0;
  for (size_t i = 0; i < kids.size(); ++i) {
    f->root_off[i] = o;
    o += kids[i].ktot;
    P.rows.insert(P.rows.end(), kids[i].rskel.begin(), kids[i].rskel.end());
    P.cols.insert(P.cols.end(), kids[i].cskel.begin(), kids[i].cskel.end());
  }
  P.m = (int)P.rows.size();
  const int m = P.m;
  if (int rc = dmalloc(f, &P.Abar, (size_t)m * m)) return rc;
  std::vector<bm_copy_desc> cp;
  std::vector<entry_job> ej;
  for (size_t a = 0; a < kids.size(); ++a) {
    const int ka = kids[a].ktot;
    const long oa = f->root_off[a];
    if (!ka) continue;
    cp.push_back(copyd(kids[a].Lam, ka, P.Abar + oa + oa * m, m, ka, ka));
    for (size_t b = 0; b < kids.size(); ++b) {
      if (b == a || !kids[b].ktot) continue;
      entry_job e = {&kids[a].rskel, &kids[b].cskel, oa + f->root_off[b] * m, m};
      ej.push_back(e);
    }
  }
  if (int rc = run_copies(f, cp)) return rc;
  return entries(f, P.Abar, ej);
}

int factor_all(bm_fds *f) {
  const int L = f->levels, n = f->leaf, N = f->n;
  f->lv.assign(L + 1, std::vector<fds_cell>());
  f->rank_sum.assign(L + 1, 0);
  f->rank_max.assign(L + 1, 0);
  // leaf cells: the three index sets (u, q, phi) of n consecutive nodes
  std::vector<fds_cell> &leaves = f->lv[L];
  leaves.resize(N / n);
  for (int i = 0; i < N / n; ++i) {
    fds_cell &c = leaves[i];
    c.level = L;
    c.index = i;
    c.node0 = i * n;
    c.nn = n;
    for (int t = 0; t < 3; ++t)
      for (int v = 0; v < n; ++v) c.rows.push_back(FDS_CODE(t, i * n + v));
    c.cols = c.rows;
    c.m = 3 * n;
  }
  // leaf diagonal blocks A_ii (eq. block_Aij) and U33^{-1}
  {
    cplx *arena = nullptr, *u33 = nullptr;
    const size_t nl = leaves.size();
    if (int rc = dmalloc(f, &arena, nl * 9 * (size_t)n * n)) return rc;
    if (int rc = dmalloc(f, &u33, nl * (size_t)n * n)) return rc;
    std::vector<entry_job> ej;
    std::vector<bm_gemm_desc> g;
    std::vector<inv_job> jobs;
    for (size_t i = 0; i < nl; ++i) {
      fds_cell &c = leaves[i];
      c.Abar = arena + i * 9 * (size_t)n * n;
      c.Ainv = u33 + i * (size_t)n * n;
      entry_job e = {&c.rows, &c.cols, (long)(i * 9 * (size_t)n * n), 3 * n};
      ej.push_back(e);
      // U33 = -[M31 M32][M13; M23] (Theorem thm:LU)
      g.push_back(gemm(n, n, 2 * n, MONE, c.Abar + 2 * n, 3 * n, c.Abar + (long)2 * n * 3 * n, 3 * n, ZERO, c.Ainv, n));
      inv_job j;
      j.A = c.Ainv;
      j.Ainv = c.Ainv;
      j.n = n;
      jobs.push_back(j);
    }
    if (int rc = entries(f, arena, ej)) return rc;
    if (int rc = run_gemms(f, g)) return rc;
    if (n > BM_FDS_GJ_MAX) return BM_E_ARG;  // the leaf inverse runs in place by Gauss-Jordan
    if (int rc = invert(f, jobs)) return rc;
  }
  for (int l = L; l >= 1; --l) {
    std::vector<fds_cell> &cells = f->lv[l];
    for (auto &c : cells) cell_geometry(f, c);
    if (l < L) {
      // A_bar^{-1} of the upper-level cells (their blocks are not needed afterwards)
      std::vector<inv_job> jobs;
      for (auto &c : cells) {
        if (int rc = dmalloc(f, &c.Ainv, (size_t)c.m * c.m)) return rc;
        inv_job j;
        j.A = c.Abar;
        j.Ainv = c.Ainv;
        j.n = c.m;
        jobs.push_back(j);
      }
      if (int rc = invert(f, jobs)) {
        FDS_FAIL(rc, "inverse of the diagonal blocks");
        return rc;
      }
    }
    if (int rc = compress_level(f, cells)) {
      FDS_FAIL(rc, "compression");
      return rc;
    }
    if (l == L) {
      if (int rc = leaf_solve_block_rhs(f, cells)) return rc;
    } else {
      std::vector<bm_gemm_desc> g;
      for (auto &c : cells) {
        if (int rc = dmalloc(f, &c.W, (size_t)c.m * c.ktot)) return rc;
        if (c.ktot) g.push_back(gemm(c.m, c.ktot, c.m, ONE, c.Ainv, c.m, c.L, c.m, ZERO, c.W, c.m));
      }
      if (int rc = run_gemms(f, g)) return rc;
    }
    if (int rc = level_lambda(f, cells)) {
      FDS_FAIL(rc, "compressed diagonal blocks (R W)^{-1}");
      return rc;
    }
    int mmax = 0;
    for (auto &c : cells) {
      f->rank_sum[l] += c.ktot;
      f->rank_max[l] = std::max(f->rank_max[l], c.ktot);
      mmax = std::max(mmax, c.m);
    }
    if (verbose())
      fprintf(stderr, "[bm_fds] level %d: %zu cells, block order <= %d, skeletons %d (max %d per cell)\n", l,
              cells.size(), mmax, f->rank_sum[l], f->rank_max[l]);
    // the root: this level's compressed system, once it is small enough to be
    // factored densely (compressing the few large cells above it would cost more
    // than it saves: a wave problem's ranks grow with the cell size)
    if (l == 1 || f->rank_sum[l] <= f->root_max) {
      f->top = l;
      if (int rc = assemble_root(f, cells)) return rc;
      break;
    }
    if (int rc = assemble_parents(f, cells, f->lv[l - 1], l - 1)) return rc;
  }
  if (verbose()) fprintf(stderr, "[bm_fds] root: the %zu cells of level %d\n", f->lv[f->top].size(), f->top);
  // root: the dense compressed system of the top level's cells
  fds_cell &root = f->lv[0][0];
  f->root_n = root.m;
  f->root_lu = root.m > BM_FDS_GJ_MAX;
  if (f->root_lu) {
    const int m = root.m;
    if (f->root_ws && f->root_ws_n < m) {
      bm_getrf_ws_destroy(f->root_ws);
      f->root_ws = nullptr;
    }
    if (!f->root_ws) {
      f->root_ws = bm_getrf_ws_create(m);
      if (!f->root_ws) return BM_E_NOMEM;
      f->root_ws_n = m;
    }
    const size_t nblk = (size_t)(m + BM_DIAG_NB - 1) / BM_DIAG_NB;
    if (int rc = dmalloc(f, &f->root_ipiv, (size_t)m)) return rc;
    if (int rc = dmalloc(f, &f->root_perm, (size_t)m)) return rc;
    if (int rc = dmalloc(f, &f->root_dinv, nblk * BM_DINV_TILES * BM_DIAG_NB * BM_DIAG_NB)) return rc;
    hipStream_t s = f->stream;
    if (int rc = bm_getrf_run(s, m, root.Abar, m, f->root_ipiv, f->dev_err, f->root_ws, 0)) return rc;
    if (int rc = bm_launch_diag_inverses(s, m, root.Abar, m, f->root_dinv)) return rc;
    if (int rc = bm_launch_perm(s, f->root_ws, m, f->root_perm)) return rc;
    int32_t h[2] = {0, 0};
    BM_HIP_TRY(hipStreamSynchronize(s));
    BM_HIP_TRY(hipMemcpy(h, f->dev_err, sizeof(h), hipMemcpyDeviceToHost));
    if (h[0] || h[1]) {
      if (verbose()) fprintf(stderr, "[bm_fds] root LU: error flag %d, zero pivot %d\n", h[0], h[1]);
      return BM_E_DEVICE;  // a bounded wait expired, or an exactly singular root
    }
    return BM_OK;
  }
  if (int rc = dmalloc(f, &root.Ainv, (size_t)root.m * root.m)) return rc;
  inv_job j;
  j.A = root.Abar;
  j.Ainv = root.Ainv;
  j.n = root.m;
  return invert(f, std::vector<inv_job>{j});
}

// ---------------------------------------------------------------------------
// Solve buffers and the solve
// ---------------------------------------------------------------------------
int alloc_solve_buffers(bm_fds *f) {
  const int L = f->levels, R = BM_FDS_RCHUNK;
  for (int l = 0; l <= L; ++l)
    for (auto &c : f->lv[l]) {
      if (int rc = dmalloc(f, &c.fb, (size_t)c.m * R)) return rc;
      if (int rc = dmalloc(f, &c.z, (size_t)c.m * R)) return rc;
      if (int rc = dmalloc(f, &c.xb, (size_t)c.m * R)) return rc;
      if (int rc = dmalloc(f, &c.t, (size_t)std::max(c.ktot, f->leaf) * R)) return rc;
      if (l == L) {
        std::vector<int> idx;
        for (int code : c.rows) idx.push_back(FDS_CODE_TYPE(code) * f->n + FDS_CODE_NODE(code));
        if (int rc = upload(f, idx, &c.gidx)) return rc;
      }
    }
  return BM_OK;
}

// offset of child ci's skeleton unknowns inside its parent's block
long child_off(bm_fds *f, int l, int ci) {
  return (ci % 2 == 0) ? 0 : f->lv[l][ci - 1].ktot;
}

int solve_chunk(bm_fds *f, int nr, const cplx *B, long ldb, cplx *X, long ldx) {
  hipStream_t s = f->stream;
  const int L = f->levels, n = f->leaf;
  // leaf right-hand sides
  for (auto &c : f->lv[L])
    if (int rc = bm_fds_rows(s, c.m, nr, c.gidx, const_cast<cplx *>(B), ldb, c.fb, c.m, 0)) return rc;
  // upward pass: z = A_bar^{-1} f_bar, g = Lambda R z (into the parent's f_bar)
  const int T = f->top;
  fds_cell &root = f->lv[0][0];
  // a cell's parent block and its offset there (the root for the top level's cells)
  auto parent = [&](int l, size_t ci) -> fds_cell & { return (l == T) ? root : f->lv[l - 1][ci / 2]; };
  auto poff = [&](int l, size_t ci) -> long { return (l == T) ? f->root_off[ci] : child_off(f, l, (int)ci); };
  for (int l = L; l >= T; --l) {
    std::vector<fds_cell> &cells = f->lv[l];
    std::vector<bm_copy_desc> cp;
    std::vector<bm_gemm_desc> g1, g2, g3;
    if (l == L) {
      // Corollary lem:for_ssm_RHS: z3 = U33^{-1}(b3 - [M31 M32][b1; b2]), [z1; z2] = [b1; b2] - [M13; M23] z3
      for (auto &c : cells) cp.push_back(copyd(c.fb, c.m, c.z, c.m, c.m, nr));
      if (int rc = run_copies(f, cp)) return rc;
      for (auto &c : cells) g1.push_back(gemm(n, nr, 2 * n, MONE, c.Abar + 2 * n, 3 * n, c.z, c.m, ONE, c.z + 2 * n, c.m));
      if (int rc = run_gemms(f, g1)) return rc;
      for (auto &c : cells) g2.push_back(gemm(n, nr, n, ONE, c.Ainv, n, c.z + 2 * n, c.m, ZERO, c.t, n));
      if (int rc = run_gemms(f, g2)) return rc;
      cp.clear();
      for (auto &c : cells) cp.push_back(copyd(c.t, n, c.z + 2 * n, c.m, n, nr));
      if (int rc = run_copies(f, cp)) return rc;
      for (auto &c : cells)
        g3.push_back(gemm(2 * n, nr, n, MONE, c.Abar + (long)2 * n * 3 * n, 3 * n, c.z + 2 * n, c.m, ONE, c.z, c.m));
      if (int rc = run_gemms(f, g3)) return rc;
    } else {
      for (auto &c : cells) g1.push_back(gemm(c.m, nr, c.m, ONE, c.Ainv, c.m, c.fb, c.m, ZERO, c.z, c.m));
      if (int rc = run_gemms(f, g1)) return rc;
    }
    std::vector<bm_gemm_desc> h1, h2;
    for (auto &c : cells)
      if (c.ktot) h1.push_back(gemm(c.ktot, nr, c.m, ONE, c.R, c.ktot, c.z, c.m, ZERO, c.t, c.ktot));
    if (int rc = run_gemms(f, h1)) return rc;
    for (size_t ci = 0; ci < cells.size(); ++ci) {
      fds_cell &c = cells[ci], &P = parent(l, ci);
      if (c.ktot) h2.push_back(gemm(c.ktot, nr, c.ktot, ONE, c.Lam, c.ktot, c.t, c.ktot, ZERO, P.fb + poff(l, ci), P.m));
    }
    if (int rc = run_gemms(f, h2)) return rc;
  }
  // root
  if (f->root_lu) {
    const int m = root.m;
    if (int rc = bm_launch_gather(s, m, nr, f->root_perm, root.fb, m, root.xb, m)) return rc;
    if (int rc = bm_trsv_reset(s, f->root_ws, m)) return rc;
    if (int rc = bm_launch_trsv(s, f->root_ws, 1, m, root.Abar, m, f->root_dinv, root.xb, m, nr, f->dev_err)) return rc;
    if (int rc = bm_launch_trsv(s, f->root_ws, 0, m, root.Abar, m, f->root_dinv, root.xb, m, nr, f->dev_err)) return rc;
  } else {
    std::vector<bm_gemm_desc> g{gemm(root.m, nr, root.m, ONE, root.Ainv, root.m, root.fb, root.m, ZERO, root.xb,
                                     root.m)};
    if (int rc = run_gemms(f, g)) return rc;
  }
  // downward pass: x_bar = z - W (g - Lambda y), y the cell's part of the parent's x_bar
  for (int l = T; l <= L; ++l) {
    std::vector<fds_cell> &cells = f->lv[l];
    std::vector<bm_copy_desc> cp;
    std::vector<bm_gemm_desc> g1, g2;
    for (size_t ci = 0; ci < cells.size(); ++ci) {
      fds_cell &c = cells[ci], &P = parent(l, ci);
      const long o = poff(l, ci);
      if (c.ktot) cp.push_back(copyd(P.fb + o, P.m, c.t, c.ktot, c.ktot, nr));  // t = g
      cp.push_back(copyd(c.z, c.m, c.xb, c.m, c.m, nr));                         // x_bar = z
    }
    if (int rc = run_copies(f, cp)) return rc;
    for (size_t ci = 0; ci < cells.size(); ++ci) {
      fds_cell &c = cells[ci], &P = parent(l, ci);
      if (c.ktot) g1.push_back(gemm(c.ktot, nr, c.ktot, MONE, c.Lam, c.ktot, P.xb + poff(l, ci), P.m, ONE, c.t, c.ktot));
    }
    if (int rc = run_gemms(f, g1)) return rc;
    for (auto &c : cells)
      if (c.ktot) g2.push_back(gemm(c.m, nr, c.ktot, MONE, c.W, c.m, c.t, c.ktot, ONE, c.xb, c.m));
    if (int rc = run_gemms(f, g2)) return rc;
  }
  for (auto &c : f->lv[L])
    if (int rc = bm_fds_rows(s, c.m, nr, c.gidx, X, ldx, c.xb, c.m, 1)) return rc;
  BM_HIP_TRY(hipStreamSynchronize(s));
  return BM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int bm_fds_create(int32_t n, const bm_fds_config *cfg, void *hip_stream, bm_fds **out) {
  if (!out) return BM_E_ARG;
  *out = nullptr;
  bm_fds_config c = {256, 128, 1e-10, 0};
  if (cfg) c = *cfg;
  if (c.root_max <= 0) c.root_max = 4096;
  if (c.leaf < 16 || c.leaf > BM_FDS_LEAF_MAX || n < 2 * c.leaf || n > 65536 || (n % c.leaf) != 0) return BM_E_ARG;
  const int p = n / c.leaf;
  if (p & (p - 1)) return BM_E_ARG;
  if (c.n_proxy < 8 || !(c.tol > 0.0) || !(c.tol < 1.0)) return BM_E_ARG;
  bm_fds *f = new (std::nothrow) bm_fds();
  if (!f) return BM_E_NOMEM;
  f->n = n;
  f->leaf = c.leaf;
  f->n_proxy = c.n_proxy;
  f->tol = c.tol;
  f->root_max = c.root_max;
  f->levels = 0;
  while ((c.leaf << f->levels) < n) ++f->levels;
  f->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&f->device) != hipSuccess) {
    delete f;
    return BM_E_HIP;
  }
  int rc = dmalloc(f, &f->geo, 8 * (size_t)n, true);
  if (!rc) rc = dmalloc(f, &f->wts, 4 * (size_t)n, true);
  if (!rc) rc = dmalloc(f, &f->dev_err, 4, true);
  if (!rc) rc = bm_launch_weights(f->stream, n, f->wts, BM_QUAD_ZETA1);
  if (!rc && hipMemsetAsync(f->dev_err, 0, 4 * sizeof(int32_t), f->stream) != hipSuccess) rc = BM_E_HIP;
  if (rc) {
    bm_fds_destroy(f);
    return rc;
  }
  memset((void *)&f->shell, 0, sizeof(f->shell));
  f->shell.n = n;
  f->shell.form = BM_MIXED;
  f->shell.nf = n;
  f->shell.stream = f->stream;
  f->shell.geo = f->geo;
  f->shell.wts = f->wts;
  f->shell.quad = BM_QUAD_ZETA1;
  *out = f;
  return BM_OK;
}

void bm_fds_destroy(bm_fds *f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->stream);
  free_factor_memory(f);
  release_spare(f, LONG_MAX);
  if (f->root_ws) bm_getrf_ws_destroy(f->root_ws);
  for (void *p : f->mem_fixed) (void)hipFree(p);
  if (f->dg) (void)hipFree(f->dg);
  if (f->dc) (void)hipFree(f->dc);
  delete f;
}

int bm_fds_factor(bm_fds *f, const bm_geometry *g, const bm_params *prm) {
  if (!f || !g || !prm || !g->x || !g->dx || !g->ddx || !g->d3x) return BM_E_ARG;
  if (int rc = bm_check_params(prm)) return rc;
  // the proxy interactions use the Hankel functions of the sector |Im k| <= Re k / 2
  if (prm->k0_im < -0.5 * prm->k0_re || prm->k1_im < -0.5 * prm->k1_re) return BM_E_ARG;
  if (hipSetDevice(f->device) != hipSuccess) return BM_E_HIP;
  BM_HIP_TRY(hipStreamSynchronize(f->stream));  // the previous factors' last readers
  free_factor_memory(f);
  const long gen_now = ++f->gen;  // this factorisation's temporaries carry gen_now
  const int n = f->n;
  f->shell.phys.k0 = cmk(prm->k0_re, prm->k0_im);
  f->shell.phys.k1 = cmk(prm->k1_re, prm->k1_im);
  f->shell.phys.beta = cmk(prm->beta_re, prm->beta_im);
  f->shell.phys.eps0 = prm->eps0;
  f->shell.phys.eps1 = prm->eps1;
  f->kmax = std::max(hypot(prm->k0_re, prm->k0_im), hypot(prm->k1_re, prm->k1_im));
  const size_t bytes = sizeof(double) * 2 * (size_t)n;
  BM_HIP_TRY(hipMemcpyAsync(f->geo, g->x, bytes, hipMemcpyDeviceToDevice, f->stream));
  BM_HIP_TRY(hipMemcpyAsync(f->geo + 2 * n, g->dx, bytes, hipMemcpyDeviceToDevice, f->stream));
  BM_HIP_TRY(hipMemcpyAsync(f->geo + 4 * n, g->ddx, bytes, hipMemcpyDeviceToDevice, f->stream));
  BM_HIP_TRY(hipMemcpyAsync(f->geo + 6 * n, g->d3x, bytes, hipMemcpyDeviceToDevice, f->stream));
  f->hx.resize(2 * (size_t)n);
  f->hdx.resize(2 * (size_t)n);
  BM_HIP_TRY(hipMemcpyAsync(f->hx.data(), f->geo, bytes, hipMemcpyDeviceToHost, f->stream));
  BM_HIP_TRY(hipMemcpyAsync(f->hdx.data(), f->geo + 2 * n, bytes, hipMemcpyDeviceToHost, f->stream));
  BM_HIP_TRY(hipStreamSynchronize(f->stream));
  BM_HIP_TRY(hipMemsetAsync(f->dev_err, 0, 4 * sizeof(int32_t), f->stream));
  int rc = factor_all(f);
  if (!rc) rc = alloc_solve_buffers(f);
  if (rc) {
    (void)hipStreamSynchronize(f->stream);
    free_factor_memory(f);
    release_spare(f, LONG_MAX);
    return rc;
  }
  BM_HIP_TRY(hipStreamSynchronize(f->stream));
  release_spare(f, gen_now);
  f->factored = true;
  return BM_OK;
}

int bm_fds_solve(bm_fds *f, int32_t nrhs, const void *B, int64_t ldb, void *X, int64_t ldx) {
  if (!f || nrhs < 0 || (nrhs > 0 && (!B || !X))) return BM_E_ARG;
  if (!f->factored) return BM_E_STATE;
  if (ldb < 3 * (int64_t)f->n || ldx < 3 * (int64_t)f->n || B == X) return BM_E_ARG;
  if (hipSetDevice(f->device) != hipSuccess) return BM_E_HIP;
  for (int r0 = 0; r0 < nrhs; r0 += BM_FDS_RCHUNK) {
    const int nr = std::min(BM_FDS_RCHUNK, nrhs - r0);
    if (int rc = solve_chunk(f, nr, (const cplx *)B + (size_t)r0 * ldb, ldb, (cplx *)X + (size_t)r0 * ldx, ldx))
      return rc;
  }
  if (f->root_lu && nrhs > 0) {  // the root's triangular solves wait (bounded) for each other's blocks
    int32_t h = 0;
    BM_HIP_TRY(hipMemcpy(&h, f->dev_err, sizeof(h), hipMemcpyDeviceToHost));
    if (h) return BM_E_DEVICE;
  }
  return BM_OK;
}

int bm_fds_rhs_plane_wave(bm_fds *f, int32_t nrhs, const double *theta_inc, void *B, int64_t ldb) {
  if (!f || nrhs < 0 || (nrhs > 0 && (!theta_inc || !B)) || ldb < 3 * (int64_t)f->n) return BM_E_ARG;
  if (!f->factored) return BM_E_STATE;
  if (nrhs == 0) return BM_OK;
  if (hipSetDevice(f->device) != hipSuccess) return BM_E_HIP;
  return bm_launch_rhs_plane_wave(&f->shell, nrhs, theta_inc, (cplx *)B, ldb);
}

int bm_fds_far_field(bm_fds *f, int32_t nrhs, const void *X, int64_t ldx, int32_t nang, const double *theta, void *F,
                     int64_t ldf) {
  if (!f || nrhs < 0 || nang < 0 || ldx < 2 * (int64_t)f->n || ldf < nang) return BM_E_ARG;
  if (nrhs > 0 && nang > 0 && (!X || !theta || !F)) return BM_E_ARG;
  if (!f->factored) return BM_E_STATE;
  if (nrhs == 0 || nang == 0) return BM_OK;
  if (hipSetDevice(f->device) != hipSuccess) return BM_E_HIP;
  return bm_launch_far_field(&f->shell, nrhs, (const cplx *)X, ldx, nang, theta, (cplx *)F, ldf);
}

int bm_fds_info(bm_fds *f, int32_t *levels, int32_t *skel_sum, int32_t *skel_max, int32_t *root_n, int64_t *bytes) {
  if (!f || !levels || !skel_sum || !skel_max || !root_n || !bytes) return BM_E_ARG;
  if (!f->factored) return BM_E_STATE;
  *levels = f->levels;
  for (int l = 0; l <= f->levels && l < 32; ++l) {
    skel_sum[l] = f->rank_sum[l];
    skel_max[l] = f->rank_max[l];
  }
  *root_n = f->root_n;
  *bytes = (int64_t)f->bytes;
  return BM_OK;
}

}  // extern "C"
