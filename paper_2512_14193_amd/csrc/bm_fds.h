// Internal declarations of the proxy-compressed fast direct solver (Sec. 4.2).
#pragma once

#include "bm_internal.h"

// rows of a column-pivoted QR target held in LDS by the step kernel
#define BM_FDS_QR_MAX_ROWS 8192
#define BM_FDS_QR_CW 32  // columns of a QR problem per workgroup

// One column-pivoted QR problem (device array of these).
struct bm_qr_prob {
  int M, C;          // target rows and columns (ld = M)
  long off;          // target at work + off
  long noff;         // per-column state at nrm2/ex2/pivd/rest + noff
  long poff;         // per-pivot state at perm/alpha + poff (kcap entries)
  int kmin, kcap;    // at least kmin pivots unless the columns run out; at most kcap
  int wg0, wgs;      // the problem's workgroups in the step launch
  long r11off, r12off;  // dense R11 (k x k) and R12 (k x (C - k)) after the passes
  // output of the interpolation matrix [I X] P^T (k x C): column c goes to row
  // o0 + i, column pos[c] of out (ld ldo), or conjugated to row pos[c], column o0 + i
  cplx *out;
  long ldo;
  int o0, conj_out;
  const int *pos;
};

// Device state arrays of a batch of problems.
struct bm_qr_state {
  double *nrm2, *ex2;   // per column: downdated and last exact squared norms
  int *pivd;            // per column: pivoted
  int *rest;            // per column: the unpivoted columns in increasing order (after the passes)
  int *perm;            // per pivot: column
  cplx *alpha;          // per pivot: R_jj
  double *bestv;        // per workgroup, two parities: best remaining squared norm
  int *bestc;           // ... and its column
  int *step;            // per problem, two parities
  int *done, *rank;     // per problem
  double *r00;          // per problem: |R_00|
};

// Explicit inverse of an n x n block in place (Gauss-Jordan, one workgroup).
struct bm_inv_desc {
  cplx *A;
  long ld;
  int n;
};

// Copy of an m x n block.
struct bm_copy_desc {
  const cplx *A;
  long lda;
  cplx *B;
  long ldb;
  int m, n;
};

int bm_fds_cpqr_prepare();
int bm_fds_cpqr_init(hipStream_t s, int nwg, const bm_qr_prob *pr, const int *wg2p, cplx *work, bm_qr_state st);
int bm_fds_cpqr_step(hipStream_t s, int nwg, const bm_qr_prob *pr, const int *wg2p, cplx *work, bm_qr_state st,
                     int L, double tol, int *active, int max_rows);
// R11, R12 of every problem into dense buffers; X = R11^{-1} R12 in place of R12 for
// ranks <= kmax_small (the others are left for a blocked solve)
int bm_fds_cpqr_finish(hipStream_t s, int nprob, const bm_qr_prob *pr, const cplx *work, bm_qr_state st, cplx *r11,
                       cplx *r12, int max_c, int kmax_small);
int bm_fds_cpqr_scatter(hipStream_t s, int nprob, const bm_qr_prob *pr, bm_qr_state st, const cplx *r12, int max_c);
int bm_fds_gj_inverse(hipStream_t s, int count, const bm_inv_desc *d_dev, int max_n, int *info_dev, int *piv_ws);
// Y = X[idx, :] (inverse = 0) or X[idx, :] = Y (inverse = 1), m rows, nr columns
int bm_fds_rows(hipStream_t s, int m, int nr, const int *idx, cplx *X, long ldx, cplx *Y, long ldy, int inverse);
int bm_fds_perm_identity(hipStream_t s, int n, const int32_t *perm, cplx *A, long ld);
int bm_fds_copy_blocks(hipStream_t s, int count, const bm_copy_desc *d_dev);
