// C ABI of the MI355X mixed Burton-Miller solver (declared in include/bm.h).
#include <math.h>
#include <string.h>

#include <new>

#include "bm_internal.h"

extern "C" {

const char *bm_strerror(int code) {
  switch (code) {
    case BM_OK: return "ok";
    case BM_E_ARG: return "invalid argument";
    case BM_E_NOMEM: return "device allocation failed";
    case BM_E_HIP: return "HIP runtime error";
    case BM_E_STATE: return "call out of order";
    case BM_E_DEVICE: return "device-side error (bounded wait expired)";
    case BM_E_NOCONV: return "iterative refinement did not reach the tolerance";
    case BM_E_BUDGET: return "request exceeds the server's device-memory budget";
    case BM_E_CANCELED: return "request canceled";
    case BM_E_TIMEOUT: return "wait timed out (request still pending)";
    case BM_E_DOMAIN: return "an argument k r of the Hankel functions lies outside the supported domain";
    default: return code > 0 ? "singular factor (info > 0)" : "unknown status";
  }
}

static void free_problem(bm_problem *p) {
  if (!p) return;
  (void)hipFree(p->geo);
  (void)hipFree(p->wts);
  (void)hipFree(p->top);
  (void)hipFree(p->bot);
  (void)hipFree(p->lu);
  (void)hipFree(p->ipiv);
  (void)hipFree(p->dinv);
  (void)hipFree(p->perm);
  (void)hipFree(p->work_g);
  (void)hipFree(p->work_p);
  (void)hipFree(p->dev_err);
  (void)hipFree(p->ir_r);
  (void)hipFree(p->ir_d);
  (void)hipFree(p->ir_norm);
  (void)hipFree(p->pipe_w);
  bm_getrf_ws_destroy(p->gws);
  for (int i = 0; i < BM_NPHASE; ++i)
    if (p->ev_created[i])
      for (int e = 0; e < BM_EV_RING; ++e) {
        (void)hipEventDestroy(p->ev[i][e][0]);
        (void)hipEventDestroy(p->ev[i][e][1]);
      }
  delete p;
}

}  // extern "C"

// Device bytes of every allocation of a problem handle: bm_create allocates
// exactly these and bm_problem_bytes adds them up (zero: not allocated).
struct bm_alloc_sizes {
  size_t geo, wts, top, bot, lu, ipiv, dinv, perm, work_g, work_p, dev_err, ir_r, ir_d, ir_norm, pipe_w;
};

static bm_alloc_sizes problem_sizes(int n, int formulation) {
  const size_t N = (size_t)n, nf = (formulation == BM_MIXED) ? N : 2 * N, c = sizeof(cplx);
  const size_t nblk = (nf + BM_DIAG_NB - 1) / BM_DIAG_NB;
  const bool mixed = formulation == BM_MIXED;
  bm_alloc_sizes z;
  z.geo = sizeof(double) * 8 * N;
  z.wts = sizeof(double) * 4 * N;
  z.top = mixed ? c * 2 * N * N : 0;
  z.bot = mixed ? c * 2 * N * N : 0;
  z.lu = c * nf * nf;
  z.ipiv = sizeof(int32_t) * nf;
  z.dinv = c * nblk * BM_DINV_TILES * BM_DIAG_NB * BM_DIAG_NB;
  z.perm = sizeof(int32_t) * nf;
  z.work_g = c * nf * BM_MAX_NRHS;
  if (mixed) {
    const size_t wp = bm_gemv_work_elems(n, 2 * n), w2 = bm_gemv_work_elems(2 * n, n);
    z.work_p = c * (wp > w2 ? wp : w2);
  } else {
    z.work_p = 0;
  }
  z.dev_err = sizeof(int32_t) * 4;
  z.ir_r = mixed ? c * 3 * N * BM_MAX_NRHS : 0;
  z.ir_d = mixed ? c * 3 * N * BM_MAX_NRHS : 0;
  z.ir_norm = mixed ? sizeof(double) * (2 * BM_MAX_NRHS + 4) : 0;  // norms, then the device refinement's state
  // split-K partials of the Schur complement computed beside the LU
  z.pipe_w = (mixed && n <= BM_PIPE_MAX_N) ? c * bm_getrf_pipe_w_elems(n) : 0;
  return z;
}

template <typename T>
static bool dev_alloc(T **ptr, size_t bytes) {
  if (bytes == 0) return true;
  return hipMalloc((void **)ptr, bytes) == hipSuccess;
}

extern "C" {

int bm_create(int32_t n, int32_t formulation, void *hip_stream, bm_problem **out) {
  if (!out) return BM_E_ARG;
  *out = nullptr;
  if (n < 8 || n > 65536 || (n % 2) != 0) return BM_E_ARG;
  if (formulation != BM_MIXED && formulation != BM_ORDINARY) return BM_E_ARG;
  bm_problem *p = new (std::nothrow) bm_problem();
  if (!p) return BM_E_NOMEM;
  memset((void *)p, 0, sizeof(*p));
  p->n = n;
  p->form = formulation;
  p->nf = (formulation == BM_MIXED) ? n : 2 * n;
  p->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free_problem(p);
    return BM_E_HIP;
  }
  const bm_alloc_sizes z = problem_sizes(n, formulation);
  bool ok = dev_alloc(&p->geo, z.geo) && dev_alloc(&p->wts, z.wts) && dev_alloc(&p->top, z.top) &&
            dev_alloc(&p->bot, z.bot) && dev_alloc(&p->lu, z.lu) && dev_alloc(&p->ipiv, z.ipiv) &&
            dev_alloc(&p->dinv, z.dinv) && dev_alloc(&p->perm, z.perm) && dev_alloc(&p->work_g, z.work_g) &&
            dev_alloc(&p->work_p, z.work_p) && dev_alloc(&p->dev_err, z.dev_err) && dev_alloc(&p->ir_r, z.ir_r) &&
            dev_alloc(&p->ir_d, z.ir_d) && dev_alloc(&p->ir_norm, z.ir_norm) && dev_alloc(&p->pipe_w, z.pipe_w);
  p->pipe_w_elems = z.pipe_w / sizeof(cplx);
  p->prec = BM_PREC_FP64;
  p->ir_tol = 1e-12;
  p->ir_maxit = 10;
  if (ok) p->gws = bm_getrf_ws_create(p->nf);
  // the Schur complement beside the LU (mixed form, FP64, N <= BM_PIPE_MAX_N); its
  // two extra streams are created by the first factorisation that uses them
  if (ok && p->gws && p->pipe_w) p->pipeline = 1;
  if (!ok || !p->gws) {
    free_problem(p);
    return BM_E_NOMEM;
  }
  if (hipMemsetAsync(p->dev_err, 0, 4 * sizeof(int32_t), p->stream) != hipSuccess) {
    free_problem(p);
    return BM_E_HIP;
  }
  p->quad = BM_QUAD_KRESS;
  int rc = bm_launch_weights(p->stream, n, p->wts, p->quad);
  if (rc) {
    free_problem(p);
    return rc;
  }
  p->state = BM_ST_CREATED;
  *out = p;
  return BM_OK;
}

void bm_destroy(bm_problem *p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  free_problem(p);
}

void bm_free(bm_problem *p) { bm_destroy(p); }

}  // extern "C"

// Phase timing: each call of a phase records an event pair in a ring of
// BM_EV_RING slots; bm_phase_times sums the pairs recorded since its last call.
void bm_phase_begin_on(bm_problem *p, int ph, hipStream_t st) {
  if (!p->profiling) return;
  if (!p->ev_created[ph]) {
    for (int e = 0; e < BM_EV_RING; ++e) {
      (void)hipEventCreate(&p->ev[ph][e][0]);
      (void)hipEventCreate(&p->ev[ph][e][1]);
    }
    p->ev_created[ph] = 1;
  }
  (void)hipEventRecord(p->ev[ph][p->ev_count[ph] % BM_EV_RING][0], st);
}

// (the end may be recorded on another stream of the device than the begin)
void bm_phase_end_on(bm_problem *p, int ph, hipStream_t st) {
  if (!p->profiling || !p->ev_created[ph]) return;
  (void)hipEventRecord(p->ev[ph][p->ev_count[ph] % BM_EV_RING][1], st);
  ++p->ev_count[ph];
}

void bm_phase_begin(bm_problem *p, int ph) { bm_phase_begin_on(p, ph, p->stream); }
void bm_phase_end(bm_problem *p, int ph) { bm_phase_end_on(p, ph, p->stream); }

static void phase_begin(bm_problem *p, int ph) { bm_phase_begin(p, ph); }
static void phase_end(bm_problem *p, int ph) { bm_phase_end(p, ph); }

extern "C" {

}  // extern "C"

int bm_check_params(const bm_params *prm) {
  if (!prm) return BM_E_ARG;
  if (!(prm->eps0 > 0.0) || !(prm->eps1 > 0.0) || !isfinite(prm->eps0) || !isfinite(prm->eps1)) return BM_E_ARG;
  if (prm->beta_im == 0.0 || !isfinite(prm->beta_re) || !isfinite(prm->beta_im)) return BM_E_ARG;
  // Re k > 0 and Im k <= Re k / 2: the sector |Im k| <= Re k / 2, or the lower half
  // plane beyond it, where the assembly checks |k| r < 6 itself (BM_E_DOMAIN)
  const double ks[2][2] = {{prm->k0_re, prm->k0_im}, {prm->k1_re, prm->k1_im}};
  for (int w = 0; w < 2; ++w)
    if (!(ks[w][0] > 0.0) || !isfinite(ks[w][0]) || !isfinite(ks[w][1]) || !(ks[w][1] <= 0.5 * ks[w][0]))
      return BM_E_ARG;
  return BM_OK;
}

extern "C" {

int bm_problem_bytes(int32_t n, int32_t formulation, int64_t *bytes) {
  if (!bytes) return BM_E_ARG;
  *bytes = 0;
  if (n < 8 || n > 65536 || (n % 2) != 0) return BM_E_ARG;
  if (formulation != BM_MIXED && formulation != BM_ORDINARY) return BM_E_ARG;
  const bm_alloc_sizes z = problem_sizes(n, formulation);
  size_t b = z.geo + z.wts + z.top + z.bot + z.lu + z.ipiv + z.dinv + z.perm + z.work_g + z.work_p + z.dev_err +
             z.ir_r + z.ir_d + z.ir_norm + z.pipe_w;
  b += bm_getrf_ws_bytes(formulation == BM_MIXED ? n : 2 * n);
  *bytes = (int64_t)b;
  return BM_OK;
}

int bm_assemble(bm_problem *p, const bm_geometry *g, const bm_params *prm) {
  if (!p || !g || !prm || !g->x || !g->dx || !g->ddx || !g->d3x) return BM_E_ARG;
  if (int rc = bm_check_params(prm)) return rc;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  p->phys.k0 = cmk(prm->k0_re, prm->k0_im);
  p->phys.k1 = cmk(prm->k1_re, prm->k1_im);
  p->phys.beta = cmk(prm->beta_re, prm->beta_im);
  p->phys.eps0 = prm->eps0;
  p->phys.eps1 = prm->eps1;
  phase_begin(p, BM_PH_ASSEMBLE);
  const size_t bytes = sizeof(double) * 2 * (size_t)p->n;
  const hipMemcpyKind kind = p->host_io ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  BM_HIP_TRY(hipMemcpyAsync(p->geo, g->x, bytes, kind, p->stream));
  BM_HIP_TRY(hipMemcpyAsync(p->geo + 2 * p->n, g->dx, bytes, kind, p->stream));
  BM_HIP_TRY(hipMemcpyAsync(p->geo + 4 * p->n, g->ddx, bytes, kind, p->stream));
  BM_HIP_TRY(hipMemcpyAsync(p->geo + 6 * p->n, g->d3x, bytes, kind, p->stream));
  bm_geometry gd = {p->geo, p->geo + 2 * p->n, p->geo + 4 * p->n, p->geo + 6 * p->n};
  int rc = bm_launch_assemble(p, &gd);
  phase_end(p, BM_PH_ASSEMBLE);
  if (rc) return rc;
  p->state = BM_ST_ASSEMBLED;
  if (p->host_io) BM_HIP_TRY(hipStreamSynchronize(p->stream));  // the host arrays may go
  return BM_OK;
}

// Host-array calls of a handle made by bm_assemble_create without BM_INPUT_DEVICE:
// device copies of the inputs, the device call, the outputs copied back, all
// complete on return.
namespace {
struct dev_buf {
  void *p = nullptr;
  ~dev_buf() { (void)hipFree(p); }
  int alloc(size_t bytes) { return (bytes == 0 || hipMalloc(&p, bytes) == hipSuccess) ? BM_OK : BM_E_NOMEM; }
};
int to_dev(bm_problem *p, dev_buf &d, const void *h, size_t rows, size_t cols, int64_t ld, size_t elem) {
  if (int rc = d.alloc(rows * cols * elem)) return rc;
  if (rows * cols == 0) return BM_OK;
  BM_HIP_TRY(hipMemcpy2DAsync(d.p, rows * elem, h, (size_t)ld * elem, rows * elem, cols, hipMemcpyHostToDevice,
                              p->stream));
  return BM_OK;
}
int to_host(bm_problem *p, void *h, int64_t ld, const dev_buf &d, size_t rows, size_t cols, size_t elem) {
  if (rows * cols == 0) return BM_OK;
  BM_HIP_TRY(hipMemcpy2DAsync(h, (size_t)ld * elem, d.p, rows * elem, rows * elem, cols, hipMemcpyDeviceToHost,
                              p->stream));
  BM_HIP_TRY(hipStreamSynchronize(p->stream));
  return BM_OK;
}
}  // namespace

int bm_assemble_create(const bm_assemble_args *a, void *hip_stream, bm_problem **out) {
  if (!out) return BM_E_ARG;
  *out = nullptr;
  if (!a || (a->flags & ~BM_INPUT_DEVICE) != 0) return BM_E_ARG;
  bm_problem *p = nullptr;
  if (int rc = bm_create(a->n, a->formulation, hip_stream, &p)) return rc;
  int rc = BM_OK;
  if (a->quadrature != BM_QUAD_KRESS) rc = bm_set_quadrature(p, a->quadrature);
  p->host_io = (a->flags & BM_INPUT_DEVICE) ? 0 : 1;
  if (!rc) rc = bm_assemble(p, &a->geometry, &a->params);
  if (!rc) rc = bm_sync(p);  // complete on return
  if (rc) {
    bm_destroy(p);
    return rc;
  }
  *out = p;
  return BM_OK;
}

static int read_dev_err(bm_problem *p, int32_t *info) {
  int32_t h[4] = {0, 0, 0, 0};
  BM_HIP_TRY(hipMemcpyAsync(h, p->dev_err, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  BM_HIP_TRY(hipStreamSynchronize(p->stream));
  if (info) *info = h[1];
  if (h[2]) return BM_E_DOMAIN;
  if (h[0]) return BM_E_DEVICE;
  return h[3] ? BM_E_NOCONV : BM_OK;  // [3]: a device-decided refinement missed its target
}

// Theorem thm:LU: U33 = -M31 M13 - M32 M23 = -[M31 M32] [M13; M23], in full, on
// the problem's stream.  Mixed precision: into a complex64 U33 that takes the first
// half of the factor storage, on the FP16 matrix cores with split operands where
// their packed planes fit in the half it leaves free, else on the FP32 ones
// (bm_solve refines against the FP64 blocks).
static int schur_product(bm_problem *p) {
  const int n = p->n;
  if (p->prec != BM_PREC_FP64) {
    const size_t half = (size_t)n * n * sizeof(cplx32);
    char *ws = (char *)p->lu + (half + 255) / 256 * 256;
    const size_t wsb = 2 * half - (size_t)(ws - (char *)p->lu);
    if (n >= BM_F16X3_MIN_N && wsb >= bm_zgemm16_ws_bytes(n, n, 16))
      return bm_launch_zgemm16(p->stream, n, n, 2 * n, cmk(-1.0, 0.0), p->bot, n, p->top, 2 * n, (cplx32 *)p->lu, n,
                               ws, wsb, nullptr);
    return bm_launch_zgemm32_c(p->stream, n, n, 2 * n, cmk(-1.0, 0.0), p->bot, n, p->top, 2 * n, cmk(0.0, 0.0),
                               (cplx32 *)p->lu, n);
  }
  return bm_launch_zgemm(p->stream, n, n, 2 * n, cmk(-1.0, 0.0), p->bot, n, p->top, 2 * n, cmk(0.0, 0.0), p->lu, n);
}

int bm_block_lu(bm_problem *p, int32_t *info) {
  if (!p) return BM_E_ARG;
  if (p->state < BM_ST_ASSEMBLED) return BM_E_STATE;
  // the ordinary matrix is factored in place: a second factorisation needs a new
  // assembly (the mixed form recomputes U33 from the blocks, which stay intact)
  if (p->form == BM_ORDINARY && p->state != BM_ST_ASSEMBLED) return BM_E_STATE;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  const int n = p->n, nf = p->nf;
  int rc = BM_OK;
  // a refinement flag left by a solve with the previous factors does not apply
  if (p->form == BM_MIXED)
    if (int rc0 = bm_launch_ir_reset(p->stream, p->ir_norm + 2 * BM_MAX_NRHS, p->dev_err + 3, 0)) return rc0;
  if (p->form == BM_MIXED && p->prec == BM_PREC_FP64 && p->pipeline) {
    if (int rc0 = bm_getrf_pipe_create(p->gws)) return rc0;
    // Theorem thm:LU: U33 = -M31 M13 - M32 M23 = -[M31 M32] [M13; M23], formed in
    // column segments beside the factorisation of the columns already formed
    phase_begin(p, BM_PH_LU);
    p->gws->prof = (p->profiling >= 2) ? p : nullptr;
    p->gws->prof_schur = p->profiling ? p : nullptr;  // the product's span in BM_PH_SCHUR
    rc = bm_getrf_schur_run(p->stream, n, cmk(-1.0, 0.0), p->bot, n, p->top, 2 * n, 2 * n, p->lu, nf, p->ipiv,
                            p->dev_err, p->gws, p->pipe_w, p->pipe_w_elems, &p->lu_segments);
    p->gws->prof = nullptr;
    p->gws->prof_schur = nullptr;
    if (!rc) rc = bm_launch_diag_inverses(p->stream, nf, p->lu, nf, p->dinv);
    if (!rc) rc = bm_launch_perm(p->stream, p->gws, nf, p->perm);
    phase_end(p, BM_PH_LU);
    if (rc) return rc;
    p->state = BM_ST_FACTORED;
    p->factored_prec = p->prec;
    if (info) return read_dev_err(p, info);
    return BM_OK;
  }
  p->lu_segments = 0;
  if (p->form == BM_MIXED) {
    // Theorem thm:LU: U33 = -M31 M13 - M32 M23 = -[M31 M32] [M13; M23]
    phase_begin(p, BM_PH_SCHUR);
    rc = schur_product(p);
    phase_end(p, BM_PH_SCHUR);
    if (rc) return rc;
    if (p->after_schur) BM_HIP_TRY(hipEventRecord(p->after_schur, p->stream));
  }
  phase_begin(p, BM_PH_LU);
  // (mixed precision: the LU of the complex64 U33, its factors stored in complex64;
  // the panels factor in FP64 registers and round on their store, the trailing
  // updates beside the next panel run on the FP32 matrix cores)
  p->gws->prof = (p->profiling >= 2) ? p : nullptr;  // per-panel timing (BM_PH_PANEL)
  const bool c64 = (p->prec != BM_PREC_FP64);
  if (c64)
    rc = bm_getrf_run_c64(p->stream, nf, (cplx32 *)p->lu, nf, p->ipiv, p->dev_err, p->gws);
  else
    rc = bm_getrf_run(p->stream, nf, p->lu, nf, p->ipiv, p->dev_err, p->gws, 0);
  p->gws->prof = nullptr;
  if (!rc)
    rc = c64 ? bm_launch_diag_inverses_c64(p->stream, nf, (const cplx32 *)p->lu, nf, p->dinv)
             : bm_launch_diag_inverses(p->stream, nf, p->lu, nf, p->dinv);
  if (!rc) rc = bm_launch_perm(p->stream, p->gws, nf, p->perm);
  phase_end(p, BM_PH_LU);
  if (rc) return rc;
  p->state = BM_ST_FACTORED;
  p->factored_prec = p->prec;
  if (info) return read_dev_err(p, info);
  return BM_OK;
}

int bm_block_lu_batch(bm_problem *const *ps, int32_t count, int32_t *info) {
  if (!ps || count < 1 || count > BM_LU_BATCH_MAX) return BM_E_ARG;
  for (int b = 0; b < count; ++b) {
    bm_problem *p = ps[b];
    if (!p || p->form != BM_MIXED) return BM_E_ARG;
    if (p->n != ps[0]->n || p->device != ps[0]->device || p->stream != ps[0]->stream || p->prec != ps[0]->prec)
      return BM_E_ARG;
    for (int c = 0; c < b; ++c)
      if (ps[c] == p) return BM_E_ARG;
    if (p->state < BM_ST_ASSEMBLED) return BM_E_STATE;
  }
  bm_problem *p0 = ps[0];
  if (hipSetDevice(p0->device) != hipSuccess) return BM_E_HIP;
  const int n = p0->n;
  const hipStream_t st = p0->stream;
  const bool c64 = (p0->prec != BM_PREC_FP64);  // the FP32 factorisation of each (complex64 U33)
  cplx *A[BM_LU_BATCH_MAX];
  cplx32 *A32[BM_LU_BATCH_MAX];
  int32_t *ipiv[BM_LU_BATCH_MAX], *err[BM_LU_BATCH_MAX];
  bm_getrf_ws *ws[BM_LU_BATCH_MAX];
  for (int b = 0; b < count; ++b) {
    bm_problem *p = ps[b];
    if (int rc0 = bm_launch_ir_reset(st, p->ir_norm + 2 * BM_MAX_NRHS, p->dev_err + 3, 0)) return rc0;
    if (int rc0 = schur_product(p)) return rc0;
    if (p->after_schur) BM_HIP_TRY(hipEventRecord(p->after_schur, st));
    p->lu_segments = 0;
    A[b] = p->lu;
    A32[b] = (cplx32 *)p->lu;
    ipiv[b] = p->ipiv;
    err[b] = p->dev_err;
    ws[b] = p->gws;
  }
  if (int rc0 = c64 ? bm_getrf_run_batch_c64(st, n, count, A32, n, ipiv, err, ws)
                    : bm_getrf_run_batch(st, n, count, A, n, ipiv, err, ws))
    return rc0;
  for (int b = 0; b < count; ++b) {
    bm_problem *p = ps[b];
    if (int rc0 = c64 ? bm_launch_diag_inverses_c64(st, n, A32[b], n, p->dinv)
                      : bm_launch_diag_inverses(st, n, p->lu, n, p->dinv))
      return rc0;
    if (int rc0 = bm_launch_perm(st, p->gws, n, p->perm)) return rc0;
    p->state = BM_ST_FACTORED;
    p->factored_prec = p->prec;
  }
  if (!info) return BM_OK;
  int status = BM_OK;
  for (int b = 0; b < count; ++b) {
    const int rc0 = read_dev_err(ps[b], &info[b]);
    if (rc0 && !status) status = rc0;
  }
  return status;
}

// One pass of the direct solve for nr <= BM_MAX_NRHS right-hand sides (X may
// not alias B).  Mixed form, Corollary lem:for_ssm_RHS.
static int solve_pass(bm_problem *p, int nr, const cplx *Bc, int64_t ldb, cplx *Xc, int64_t ldx) {
  const int n = p->n, nf = p->nf;
  const int rows = (p->form == BM_MIXED) ? 3 * n : 2 * n;
  BM_HIP_TRY(hipMemcpy2DAsync(Xc, sizeof(cplx) * ldx, Bc, sizeof(cplx) * ldb, sizeof(cplx) * rows, nr,
                              hipMemcpyDeviceToDevice, p->stream));
  cplx *X3 = (p->form == BM_MIXED) ? Xc + 2 * n : Xc;
  cplx *Y = p->work_g;  // nf x nr, ld nf
  int rc;
  if (p->form == BM_MIXED) {
    // c = b3 - M31 b1 - M32 b2 = b3 - Bot [b1; b2]
    rc = bm_launch_gemv_sub(p->stream, n, 2 * n, nr, p->bot, n, Xc, ldx, X3, ldx, p->work_p);
    if (rc) return rc;
  }
  rc = bm_launch_gather(p->stream, nf, nr, p->perm, X3, ldx, Y, nf);
  if (!rc) rc = bm_trsv_reset(p->stream, p->gws, nf);
  if (p->factored_prec != BM_PREC_FP64) {  // complex64 factors
    const cplx32 *lu32 = (const cplx32 *)p->lu;
    if (!rc) rc = bm_launch_trsv_c64(p->stream, p->gws, 1, nf, lu32, nf, p->dinv, Y, nf, nr, p->dev_err);
    if (!rc) rc = bm_launch_trsv_c64(p->stream, p->gws, 0, nf, lu32, nf, p->dinv, Y, nf, nr, p->dev_err);
  } else {
    if (!rc) rc = bm_launch_trsv(p->stream, p->gws, 1, nf, p->lu, nf, p->dinv, Y, nf, nr, p->dev_err);
    if (!rc) rc = bm_launch_trsv(p->stream, p->gws, 0, nf, p->lu, nf, p->dinv, Y, nf, nr, p->dev_err);
  }
  if (rc) return rc;
  BM_HIP_TRY(hipMemcpy2DAsync(X3, sizeof(cplx) * ldx, Y, sizeof(cplx) * nf, sizeof(cplx) * nf, nr,
                              hipMemcpyDeviceToDevice, p->stream));
  if (p->form == BM_MIXED) {
    // x1 = b1 - M13 z3, x2 = b2 - M23 z3:  [x1; x2] = [b1; b2] - Top z3
    rc = bm_launch_gemv_sub(p->stream, 2 * n, n, nr, p->top, 2 * n, Y, nf, Xc, ldx, p->work_p);
    if (rc) return rc;
  }
  return BM_OK;
}

// Residual r = b - A x of the mixed system with the FP64 blocks:
//   [r1; r2] = [b1; b2] - [x1; x2] - Top x3,   r3 = b3 - Bot [x1; x2].
// Returns max_j ||r_j|| / ||b_j|| (synchronises the stream).
// The residual R = b - A x and its column norms (ir_norm), enqueued only.
static int residual_enqueue(bm_problem *p, int nr, const cplx *Bc, int64_t ldb, const cplx *Xc, int64_t ldx) {
  const int n = p->n, rows = 3 * n;
  cplx *R = p->ir_r;
  int rc = bm_launch_ir_prep(p->stream, rows, 2 * n, nr, Bc, ldb, Xc, ldx, R, rows);
  if (!rc) rc = bm_launch_gemv_sub(p->stream, 2 * n, n, nr, p->top, 2 * n, Xc + 2 * n, ldx, R, rows, p->work_p);
  if (!rc) rc = bm_launch_gemv_sub(p->stream, n, 2 * n, nr, p->bot, n, Xc, ldx, R + 2 * n, rows, p->work_p);
  if (!rc) rc = bm_launch_colnorms(p->stream, rows, nr, R, rows, Bc, ldb, p->ir_norm);
  return rc;
}

static int residual(bm_problem *p, int nr, const cplx *Bc, int64_t ldb, const cplx *Xc, int64_t ldx, double *relres) {
  if (int rc = residual_enqueue(p, nr, Bc, ldb, Xc, ldx)) return rc;
  double h[2 * BM_MAX_NRHS];
  BM_HIP_TRY(hipMemcpyAsync(h, p->ir_norm, sizeof(double) * 2 * nr, hipMemcpyDeviceToHost, p->stream));
  BM_HIP_TRY(hipStreamSynchronize(p->stream));
  double worst = 0.0;
  for (int j = 0; j < nr; ++j) {
    const double rj = sqrt(h[2 * j]), bj = sqrt(h[2 * j + 1]);
    const double q = (bj > 0.0) ? rj / bj : rj;
    if (!(q <= worst)) worst = q;  // NaN propagates
  }
  *relres = worst;
  return BM_OK;
}

int bm_solve(bm_problem *p, int32_t nrhs, const void *Bv, int64_t ldb, void *Xv, int64_t ldx) {
  if (!p || nrhs < 0 || (nrhs > 0 && (!Bv || !Xv))) return BM_E_ARG;
  if (p->state < BM_ST_FACTORED) return BM_E_STATE;
  const int n = p->n;
  const int rows = (p->form == BM_MIXED) ? 3 * n : 2 * n;
  if (ldb < rows || ldx < rows) return BM_E_ARG;
  if (Bv == Xv) return BM_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (p->host_io) {
    if (nrhs == 0) return BM_OK;
    dev_buf db, dx;
    if (int rc = to_dev(p, db, Bv, rows, nrhs, ldb, sizeof(cplx))) return rc;
    if (int rc = dx.alloc(sizeof(cplx) * rows * (size_t)nrhs)) return rc;
    p->host_io = 0;
    int rc = bm_solve(p, nrhs, db.p, rows, dx.p, rows);
    p->host_io = 1;
    if (!rc) rc = to_host(p, Xv, ldx, dx, rows, nrhs, sizeof(cplx));
    return rc;
  }
  const cplx *B = (const cplx *)Bv;
  cplx *X = (cplx *)Xv;
  const bool refine = (p->factored_prec == BM_PREC_MIXED);
  const bool refine_dev = (p->factored_prec == BM_PREC_MIXED_DEVICE);
  double *ctl = p->ir_norm + 2 * BM_MAX_NRHS;  // the device refinement's state
  int status = BM_OK;
  p->ir_iters = 0;
  p->ir_relres = 0.0;
  p->ir_dev_stats = refine_dev;
  phase_begin(p, BM_PH_SOLVE);
  if (refine_dev) {
    if (int rc = bm_launch_ir_reset(p->stream, ctl, p->dev_err + 3, 0)) return rc;
  }
  for (int r0 = 0; r0 < nrhs; r0 += BM_MAX_NRHS) {
    const int nr = (nrhs - r0 < BM_MAX_NRHS) ? nrhs - r0 : BM_MAX_NRHS;
    const cplx *Bc = B + (size_t)r0 * ldb;
    cplx *Xc = X + (size_t)r0 * ldx;
    int rc = solve_pass(p, nr, Bc, ldb, Xc, ldx);
    if (rc) return rc;
    if (refine_dev) {
      // exactly ir_maxit passes, each applied only while the previous residual
      // test fails; the tests are kernels (nothing waits for the host)
      rc = bm_launch_ir_reset(p->stream, ctl, p->dev_err + 3, 1);
      for (int it = 0; !rc && it < p->ir_maxit; ++it) {
        rc = residual_enqueue(p, nr, Bc, ldb, Xc, ldx);
        if (!rc) rc = bm_launch_ir_check(p->stream, nr, p->ir_norm, p->ir_tol, ctl, p->dev_err + 3, 0);
        if (!rc) rc = solve_pass(p, nr, p->ir_r, rows, p->ir_d, rows);
        if (!rc) rc = bm_launch_axpy_if(p->stream, rows, nr, p->ir_d, rows, Xc, ldx, ctl);
      }
      if (!rc) rc = residual_enqueue(p, nr, Bc, ldb, Xc, ldx);
      if (!rc) rc = bm_launch_ir_check(p->stream, nr, p->ir_norm, p->ir_tol, ctl, p->dev_err + 3, 1);
      if (rc) return rc;
    }
    if (refine) {
      // FP64 iterative refinement: x += A_f^{-1} (b - A x) with the FP64 blocks in
      // the residual and the mixed-precision factors in the correction
      double rr = 0.0;
      int it = 0;
      for (;;) {
        rc = residual(p, nr, Bc, ldb, Xc, ldx, &rr);
        if (rc) return rc;
        if (rr <= p->ir_tol || it >= p->ir_maxit) break;
        rc = solve_pass(p, nr, p->ir_r, rows, p->ir_d, rows);
        if (!rc) rc = bm_launch_axpy(p->stream, rows, nr, p->ir_d, rows, Xc, ldx);
        if (rc) return rc;
        ++it;
      }
      if (it > p->ir_iters) p->ir_iters = it;
      if (!(rr <= p->ir_relres)) p->ir_relres = rr;
      if (!(rr <= p->ir_tol)) status = BM_E_NOCONV;
    }
  }
  phase_end(p, BM_PH_SOLVE);
  return status;
}

int bm_set_precision(bm_problem *p, int32_t precision, double tol, int32_t max_iter) {
  if (!p) return BM_E_ARG;
  if (precision != BM_PREC_FP64 && precision != BM_PREC_MIXED && precision != BM_PREC_MIXED_DEVICE) return BM_E_ARG;
  if (precision != BM_PREC_FP64 && p->form != BM_MIXED) return BM_E_ARG;
  if (!(tol > 0.0) || max_iter < 0) return BM_E_ARG;
  p->prec = precision;
  p->ir_tol = tol;
  p->ir_maxit = max_iter;
  return BM_OK;
}

int bm_set_quadrature(bm_problem *p, int32_t quadrature) {
  if (!p) return BM_E_ARG;
  if (quadrature != BM_QUAD_KRESS && quadrature != BM_QUAD_ZETA1 && quadrature != BM_QUAD_ZETA31) return BM_E_ARG;
  if (quadrature == BM_QUAD_ZETA31 && p->n < 32) return BM_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (int rc = bm_launch_weights(p->stream, p->n, p->wts, quadrature)) return rc;
  p->quad = quadrature;
  if (p->state > BM_ST_CREATED) p->state = BM_ST_CREATED;  // blocks of the old rule are stale
  return BM_OK;
}

int bm_set_lu_overlap(bm_problem *p, int32_t on) {
  if (!p || (on != 0 && on != 1)) return BM_E_ARG;
  if (on && (!p->pipe_w || !p->gws)) return BM_E_ARG;
  p->pipeline = on;
  return BM_OK;
}

int bm_lu_overlap_info(bm_problem *p, int32_t *enabled, int32_t *segments) {
  if (!p || !enabled || !segments) return BM_E_ARG;
  *enabled = p->pipeline;
  *segments = p->lu_segments;
  return BM_OK;
}

int bm_refine_stats(bm_problem *p, int32_t *iterations, double *rel_residual) {
  if (!p || !iterations || !rel_residual) return BM_E_ARG;
  if (p->ir_dev_stats) {  // the device refinement's record of the latest solve
    double h[4];
    BM_HIP_TRY(hipMemcpyAsync(h, p->ir_norm + 2 * BM_MAX_NRHS, sizeof(h), hipMemcpyDeviceToHost, p->stream));
    BM_HIP_TRY(hipStreamSynchronize(p->stream));
    p->ir_iters = (int)h[3];
    p->ir_relres = h[2];
    p->ir_dev_stats = 0;
  }
  *iterations = p->ir_iters;
  *rel_residual = p->ir_relres;
  return BM_OK;
}

int bm_rhs_plane_wave(bm_problem *p, int32_t nrhs, const double *theta_inc, void *B, int64_t ldb) {
  if (!p || nrhs < 0 || (nrhs > 0 && (!theta_inc || !B))) return BM_E_ARG;
  if (p->state < BM_ST_ASSEMBLED) return BM_E_STATE;
  const int rows = (p->form == BM_MIXED) ? 3 * p->n : 2 * p->n;
  if (ldb < rows) return BM_E_ARG;
  if (nrhs == 0) return BM_OK;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (p->host_io) {
    dev_buf dt, dbuf;
    if (int rc = to_dev(p, dt, theta_inc, nrhs, 1, nrhs, sizeof(double))) return rc;
    if (int rc = dbuf.alloc(sizeof(cplx) * rows * (size_t)nrhs)) return rc;
    int rc = bm_launch_rhs_plane_wave(p, nrhs, (const double *)dt.p, (cplx *)dbuf.p, rows);
    if (!rc) rc = to_host(p, B, ldb, dbuf, rows, nrhs, sizeof(cplx));
    return rc;
  }
  return bm_launch_rhs_plane_wave(p, nrhs, theta_inc, (cplx *)B, ldb);
}

int bm_far_field(bm_problem *p, int32_t nrhs, const void *X, int64_t ldx, int32_t nang, const double *theta,
                 void *F, int64_t ldf) {
  if (!p || nrhs < 0 || nang < 0) return BM_E_ARG;
  if (nrhs > 0 && nang > 0 && (!X || !theta || !F)) return BM_E_ARG;
  if (p->state < BM_ST_ASSEMBLED) return BM_E_STATE;
  if (ldx < 2 * p->n || ldf < nang) return BM_E_ARG;
  if (nrhs == 0 || nang == 0) return BM_OK;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (p->host_io) {
    const size_t rx = 2 * (size_t)p->n;  // the traces [u; q] the far field reads
    dev_buf dxb, dt, df;
    if (int rc = to_dev(p, dxb, X, rx, nrhs, ldx, sizeof(cplx))) return rc;
    if (int rc = to_dev(p, dt, theta, nang, 1, nang, sizeof(double))) return rc;
    if (int rc = df.alloc(sizeof(cplx) * nang * (size_t)nrhs)) return rc;
    p->host_io = 0;
    int rc = bm_far_field(p, nrhs, dxb.p, (int64_t)rx, nang, (const double *)dt.p, df.p, nang);
    p->host_io = 1;
    if (!rc) rc = to_host(p, F, ldf, df, nang, nrhs, sizeof(cplx));
    return rc;
  }
  phase_begin(p, BM_PH_FAR);
  int rc = bm_launch_far_field(p, nrhs, (const cplx *)X, ldx, nang, theta, (cplx *)F, ldf);
  phase_end(p, BM_PH_FAR);
  return rc;
}

int bm_copy_blocks(bm_problem *p, void *a, int64_t lda, void *b, int64_t ldb) {
  if (!p || !a) return BM_E_ARG;
  if (p->state != BM_ST_ASSEMBLED && !(p->form == BM_MIXED && p->state == BM_ST_FACTORED)) return BM_E_STATE;
  const size_t N = (size_t)p->n;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (p->form == BM_MIXED) {
    if (!b || lda < (int64_t)(2 * N) || ldb < (int64_t)N) return BM_E_ARG;
    BM_HIP_TRY(hipMemcpy2DAsync(a, sizeof(cplx) * lda, p->top, sizeof(cplx) * 2 * N, sizeof(cplx) * 2 * N, N,
                                hipMemcpyDeviceToDevice, p->stream));
    BM_HIP_TRY(hipMemcpy2DAsync(b, sizeof(cplx) * ldb, p->bot, sizeof(cplx) * N, sizeof(cplx) * N, 2 * N,
                                hipMemcpyDeviceToDevice, p->stream));
  } else {
    if (lda < (int64_t)(2 * N)) return BM_E_ARG;
    BM_HIP_TRY(hipMemcpy2DAsync(a, sizeof(cplx) * lda, p->lu, sizeof(cplx) * 2 * N, sizeof(cplx) * 2 * N, 2 * N,
                                hipMemcpyDeviceToDevice, p->stream));
  }
  return BM_OK;
}

int bm_copy_factors(bm_problem *p, void *lu, int64_t ld, int32_t *ipiv) {
  if (!p || !lu || !ipiv) return BM_E_ARG;
  if (p->state < BM_ST_FACTORED) return BM_E_STATE;
  const size_t nf = (size_t)p->nf;
  if (ld < (int64_t)nf) return BM_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  if (p->factored_prec != BM_PREC_FP64) {  // complex64 factors, widened
    if (int rc = bm_launch_widen(p->stream, (int)nf, (int)nf, (const cplx32 *)p->lu, (int64_t)nf, (cplx *)lu, ld))
      return rc;
  } else {
    BM_HIP_TRY(hipMemcpy2DAsync(lu, sizeof(cplx) * ld, p->lu, sizeof(cplx) * nf, sizeof(cplx) * nf, nf,
                                hipMemcpyDeviceToDevice, p->stream));
  }
  BM_HIP_TRY(hipMemcpyAsync(ipiv, p->ipiv, sizeof(int32_t) * nf, hipMemcpyDeviceToDevice, p->stream));
  return BM_OK;
}

int bm_sync(bm_problem *p) {
  if (!p) return BM_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return BM_E_HIP;
  return read_dev_err(p, nullptr);
}

int bm_set_profiling(bm_problem *p, int32_t enable) {
  if (!p) return BM_E_ARG;
  p->profiling = (enable >= 2) ? 2 : (enable ? 1 : 0);
  return BM_OK;
}

int bm_phase_times(bm_problem *p, double *ms, int32_t *count, int32_t n_phase) {
  if (!p || !ms || !count || n_phase < 0 || n_phase > BM_NPHASE) return BM_E_ARG;
  BM_HIP_TRY(hipStreamSynchronize(p->stream));
  for (int i = 0; i < n_phase; ++i) {
    const int c = p->ev_count[i] < BM_EV_RING ? p->ev_count[i] : BM_EV_RING;
    double tot = 0.0;
    for (int e = 0; e < c; ++e) {
      float f = 0.0f;
      if (hipEventElapsedTime(&f, p->ev[i][e][0], p->ev[i][e][1]) == hipSuccess) tot += f;
    }
    ms[i] = tot;
    count[i] = c;
    p->ev_count[i] = 0;
  }
  return BM_OK;
}

int bm_zgemm(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha, const void *A, int64_t lda,
             const void *B, int64_t ldb, const double *beta, void *C, int64_t ldc) {
  if (m < 0 || n < 0 || k < 0 || !alpha || !beta) return BM_E_ARG;
  if (m == 0 || n == 0) return BM_OK;
  if (!C || (k > 0 && (!A || !B))) return BM_E_ARG;
  if (lda < m || ldb < k || ldc < m) return BM_E_ARG;
  return bm_launch_zgemm((hipStream_t)hip_stream, m, n, k, cmk(alpha[0], alpha[1]), (const cplx *)A, lda,
                         (const cplx *)B, ldb, cmk(beta[0], beta[1]), (cplx *)C, ldc);
}

int bm_zgemm_f32(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha, const void *A,
                 int64_t lda, const void *B, int64_t ldb, const double *beta, void *C, int64_t ldc) {
  if (m < 0 || n < 0 || k < 0 || !alpha || !beta) return BM_E_ARG;
  if (m == 0 || n == 0) return BM_OK;
  if (!C || (k > 0 && (!A || !B))) return BM_E_ARG;
  if (lda < m || ldb < k || ldc < m) return BM_E_ARG;
  return bm_launch_zgemm32((hipStream_t)hip_stream, m, n, k, cmk(alpha[0], alpha[1]), (const cplx *)A, lda,
                           (const cplx *)B, ldb, cmk(beta[0], beta[1]), (cplx *)C, ldc);
}

int bm_zgemm_f16x3(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha, const void *A,
                   int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, void *ws, int64_t ws_bytes) {
  if (m < 0 || n < 0 || k < 0 || !alpha || ws_bytes < 0) return BM_E_ARG;
  if (m == 0 || n == 0) return BM_OK;
  if (!C || (k > 0 && (!A || !B)) || !ws) return BM_E_ARG;
  if (lda < m || ldb < k || ldc < m) return BM_E_ARG;
  return bm_launch_zgemm16((hipStream_t)hip_stream, m, n, k, cmk(alpha[0], alpha[1]), (const cplx *)A, lda,
                           (const cplx *)B, ldb, (cplx32 *)C, ldc, ws, (size_t)ws_bytes, nullptr);
}

int64_t bm_zgemm_f16x3_ws_bytes(int32_t m, int32_t n, int32_t k, int32_t k_chunk) {
  if (m < 0 || n < 0 || k < 0 || k_chunk < 1) return -1;
  return (int64_t)bm_zgemm16_ws_bytes(m, n, k_chunk < k ? k_chunk : (k > 0 ? k : 1));
}

int bm_zgetrf(void *hip_stream, int32_t n, void *A, int64_t lda, int32_t *ipiv, int32_t *info) {
  if (n < 0 || lda < n || (n > 0 && (!A || !ipiv))) return BM_E_ARG;
  if (n == 0) {
    if (info) *info = 0;
    return BM_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  bm_getrf_ws *w = bm_getrf_ws_create(n);
  int32_t *dev_err = nullptr;
  if (!w || hipMalloc(&dev_err, 2 * sizeof(int32_t)) != hipSuccess) {
    bm_getrf_ws_destroy(w);
    return BM_E_NOMEM;
  }
  int rc = bm_getrf_run(s, n, (cplx *)A, lda, ipiv, dev_err, w, 0);
  int32_t h[2] = {0, 0};
  if (hipMemcpyAsync(h, dev_err, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = rc ? rc : BM_E_HIP;
  (void)hipFree(dev_err);
  bm_getrf_ws_destroy(w);
  if (rc) return rc;
  if (info) *info = h[1];
  return h[0] ? BM_E_DEVICE : BM_OK;
}

}  // extern "C"
