// Blocked right-looking LU with partial pivoting for gfx950 (complex FP64).
//
// Used for U33 = -M31 M13 - M32 M23 (Theorem thm:LU) and, as the comparator, for
// the 2N x 2N ordinary matrix.  Per panel of jb <= 64 columns starting at column j:
//
//  1. panel_kernel (P workgroups, all resident at once): the (n - j) x jb panel
//     is held in LDS for the whole panel, 64 or 128 consecutive rows per
//     workgroup.  In each workgroup one wavefront runs the chain that decides the
//     pivots (receive the candidates of column c, select, exchange rows, scale
//     column c, update column c + 1, publish the candidate of column c + 1) with
//     no workgroup barrier, and the other wavefronts apply the rest of each rank-1
//     update one step behind it.  The candidate of a workgroup (value, row and the
//     whole candidate row) goes to an exchange record; every workgroup reads all
//     P records and picks the same winner: one cross-workgroup round trip per
//     column.
//  2. swap_trsm_kernel: the panel's row interchanges, composed into one permutation
//     of at most 2 jb rows, on every column outside the panel; for the columns right
//     of the panel also U12 = L11^{-1} A12 by forward substitution, one or two
//     columns per wavefront with lane = row.
//  3. trailing update A22 -= L21 U12 with the MFMA GEMM.
//  Steps 2 and 3 run first for the next panel's columns only; for all other
//  columns they run on a second stream while the next panel is factored
//  (lookahead of depth one).  Beside the Schur product (below), a panel of 64
//  rows per workgroup and at least 10 workgroups does steps 2 and 3 for its own
//  columns itself, before its chain starts (the fused form of panel_kernel).
//
// Cross-workgroup data is written with agent-scope stores and read with agent-scope
// loads, which are coherent across the XCDs' separate L2 caches.  Every wait is
// bounded: on expiry the kernel raises the device error flag and runs to completion.
#include <cstring>
#include <mutex>

#include "bm_internal.h"
#include "bm_trinv.h"

// ---------------------------------------------------------------------------
// 1. panel factorisation
//
// Exchange protocol: for column c every workgroup g writes one record
//   slots[c][g] = { (value, row), candidate row (jb complex values) }
// and the owner of row j + c also writes that row after the P records.  Slots are
// filled with an all-ones bit pattern before the panel starts (a NaN the
// arithmetic never produces), each word is written exactly once with an
// agent-scope store, and readers poll each word with agent-scope loads until it
// differs from the pattern.  So the data itself is the synchronisation: no fence,
// no counter, one round trip per column (a reader takes the headers, then the
// winner's row and the diagonal row, written right after the header).
// ---------------------------------------------------------------------------
#define PANEL_PMAX 256            // max workgroups of a panel launch
#define SENT 0xFFFFFFFFFFFFFFFFULL  // empty exchange word (all ones)
#define SNT 448                   // threads per panel workgroup: one chain + SNB bulk wavefronts
#define SNB 6
#define PANEL_RPL1_PMAX 32        // 64 rows per workgroup while P stays within this, else 128
#define PANEL_LDS(rpl) ((size_t)LU_NB * (64 * (rpl) + 1) * sizeof(cplx))
// LDS requested by every panel launch: more than 160 KB minus any GEMM workgroup's
// share, so that no workgroup of the concurrent trailing update lands on a CU that
// runs a panel workgroup (the chain wavefront would lose issue slots)
#define PANEL_LDS_ALLOC PANEL_LDS(2)

// Slot buffer layout: per column c, the P records of rec = jb + 1 complex values
// (candidate row, then its value and row index) followed by the diagonal row, and,
// after all columns' records, the P headers (value, row) of every column side by
// side (16 bytes each: one poll instruction of the chain reads P / 8 cache lines).
#define SLOT_REC_ELEMS ((size_t)LU_NB * (PANEL_PMAX * (LU_NB + 1) + LU_NB))
#define SLOT_HDR ((int)SLOT_REC_ELEMS)  // header of column c, workgroup g: SLOT_HDR + c P + g
// after the headers, the U12 block (LU_NB x LU_NB, column-major) of a panel that
// applies the previous panel's update to its own columns (the fused form below)
#define SLOT_U12 ((int)(SLOT_REC_ELEMS + (size_t)LU_NB * PANEL_PMAX))
#define SLOT_ELEMS ((size_t)SLOT_U12 + (size_t)LU_NB * LU_NB)  // complex values per slot buffer

// 16-byte agent-coherent loads and stores of the exchange records: buffer
// instructions with the sc1 cache-policy bit (agent scope on gfx94x / gfx950).
// A record word reads as empty while either 8-byte half still holds the pattern.
typedef int bm_v4i __attribute__((ext_vector_type(4)));
#define BM_BUF_DW3 0x00020000  // buffer descriptor word 3 for raw (untyped) access on gfx9
#define BM_CPOL_SC1 16
__device__ inline __amdgpu_buffer_rsrc_t rec_rsrc(const cplx *slots) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)slots, 0, (int)(SLOT_ELEMS * sizeof(cplx)), BM_BUF_DW3);
}
__device__ inline bm_v4i rec_load(__amdgpu_buffer_rsrc_t r, int elem) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, elem * (int)sizeof(cplx), 0, BM_CPOL_SC1);
}
__device__ inline void rec_store(__amdgpu_buffer_rsrc_t r, int elem, cplx v) {
  bm_v4i x;
  x[0] = __double2loint(v.x);
  x[1] = __double2hiint(v.x);
  x[2] = __double2loint(v.y);
  x[3] = __double2hiint(v.y);
  __builtin_amdgcn_raw_buffer_store_b128(x, r, elem * (int)sizeof(cplx), 0, BM_CPOL_SC1);
}
__device__ inline bool rec_empty(bm_v4i v) { return (v[0] & v[1]) == -1 || (v[2] & v[3]) == -1; }
__device__ inline cplx rec_value(bm_v4i v) { return cmk(__hiloint2double(v[1], v[0]), __hiloint2double(v[3], v[2])); }

// one record value, polled until written (bounded)
__device__ inline cplx rec_poll(__amdgpu_buffer_rsrc_t r, int elem, int32_t *dev_err, bool &ok) {
  bm_v4i v = rec_load(r, elem);
  const unsigned long long t0 = wall_clock64();
  while (rec_empty(v)) {
    if (!ok || wait_expired(t0)) {
      if (ok) atomicOr(dev_err, 1);
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    v = rec_load(r, elem);
  }
  return rec_value(v);
}

// Wave-wide maximum of a double by DPP row operations (a few ALU cycles per step,
// no LDS round trip); NaN entries are ignored.  Must be called with all 64 lanes
// active.  The result is broadcast from lane 63.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(rhi, rlo);
}

__device__ inline double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));        // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));        // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));       // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));       // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v));  // row_bcast15 into rows 1 and 3
  v = fmax(v, dpp_f64<0x143, 0xC>(v));  // row_bcast31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// First lane holding the wave maximum of v (>= 0), or -1 if no lane holds a value
// >= 0.  Lanes are in row order, so ties resolve to the smallest row.
__device__ inline int wave_argmax_first(double v, double &vmax) {
  const double m = wave_max_f64(v);
  vmax = m;
  if (!(m >= 0.0)) return -1;
  const unsigned long long mask = __ballot(v == m);
  return mask ? (int)__ffsll((long long)mask) - 1 : -1;
}

__device__ inline int wave_min_int(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off));
  return x;
}

// value of lane l (wave-uniform l) in every lane
__device__ inline double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ inline cplx readlane_c(cplx v, int l) { return cmk(readlane_f64(v.x, l), readlane_f64(v.y, l)); }

// component-wise select (keeps register arrays out of memory)
__device__ inline cplx csel(bool c, cplx a, cplx b) { return cmk(c ? a.x : b.x, c ? a.y : b.y); }

// 1/u for the pivot: the larger component is scaled to [0.5, 1) by an exact power
// of two, then conj(u) / |u|^2 with a Newton-refined hardware reciprocal
__device__ inline cplx pivot_recip(cplx u) {
  int e = 0;
  (void)frexp(fmax(fabs(u.x), fabs(u.y)), &e);
  const cplx us = cmk(ldexp(u.x, -e), ldexp(u.y, -e));
  const double d = fma(us.x, us.x, us.y * us.y);
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  r = ldexp(r, -e);
  return cmk(us.x * r, -us.y * r);
}

// Panel factorisation with split roles.  A workgroup holds RPW = 64 RPL rows of
// the panel in LDS (column-major, padded stride LDP).  Wavefront 0 runs the chain
// that decides the pivots, without workgroup barriers; wavefronts 1 .. SNB apply
// the bulk of each rank-1 update one step behind it.  Per column c:
//   wavefront 0: receives the P record headers of column c, selects the winner p
//   and fetches its row and the diagonal row; in registers it exchanges rows
//   j + c and p, scales column c (the multipliers l_r = a_rc / u_c), updates
//   column c + 1 and finds the workgroup's candidate for it, whose header it
//   publishes at once (the header is what every reader waits for); then come
//   the candidate and diagonal rows of the record (from the registers and the LDS
//   as it stands, completed on the fly for columns > c + 1), the LDS writes of the
//   step, and pivot c is released to the bulk wavefronts; it also applies pivot
//   c to column c + 2 and keeps that column in registers, so the next step
//   starts without touching LDS;
//   wavefronts 1 .. SNB: subtract l_r u_cc from columns cc >= c + 3 and count
//   themselves done; wavefront 0 waits for that count before it writes rows or
//   reads columns of the next step.
// Exchange layout per column c (rs = record stride, cstride = complex values per column):
//   slots[c * cstride + g * rs]  record of workgroup g: (value, row), then the row
//   slots[c * cstride + P * rs]  the diagonal row j + c, by its owner
//   slots[SLOT_HDR + c * P + g]  the header (value, row) of workgroup g when packed
typedef double pdbl4 __attribute__((ext_vector_type(4)));
__device__ inline pdbl4 pmfma16(double a, double b, pdbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FUSE: the panel first applies the previous panel's update to its own columns
// (what the separate interchange/TRSM and k = 64 update launches do otherwise):
// the previous panel (columns j0 .. j0 + 63, interchange list swp0) gives
//   U12 = L11^{-1} (its interchanged rows j0 .. j0 + 63 of these columns),
//   each row r >= j:  a_r = (row sigma(r) of these columns) - L(r, j0..) U12,
// sigma the interchanges' row sources.  Every workgroup solves the columns
// c = g (mod P) of U12 (lane = row, one column per wavefront) and publishes them
// in the slot buffer's U12 block with the exchange protocol (agent-scope stores
// over the empty pattern, polled by the readers); every workgroup then reads all
// of U12 and forms its rows' update on the FP64 matrix cores.  Rows j0 .. j0 + 63
// of these columns (U12 itself) are written back by workgroup 0 at the end, when
// every workgroup has long finished reading the old values (it has published its
// candidate of column 0, which workgroup 0 waited for).  RPL = 1 and P >= 10 only.
// (BAT: a batch of problems, blockIdx.y selecting the problem's matrix, pivots,
// flags, exchange slots and interchange list from bb)
template <int RPL, bool FUSE, class T, bool BAT = false>
__global__ __launch_bounds__(SNT) void panel_kernel(int N, T *A, long lda, int j, int jb, int P, int32_t *ipiv,
                                                    int32_t *dev_err, cplx *slots, cplx *next_slots, int next_P,
                                                    int next_jb, int32_t *swp, int j0, const int32_t *swp0,
                                                    bm_lu_batch bb) {
  if constexpr (BAT) {
    static_assert(!FUSE, "batched panels: no fused update");
    const int b = blockIdx.y;
    A = (T *)bb.A[b];
    ipiv = bb.ipiv[b];
    dev_err = bb.err[b];
    slots = bb.cur[b];
    next_slots = bb.nxt[b];
    swp = bb.swp[b];
  }
  constexpr int RPW = 64 * RPL;  // rows per workgroup
  constexpr int LDP = RPW + 1;   // column stride of the LDS panel (odd: conflict-free row reads)
  extern __shared__ cplx pan[];  // jb x LDP
  __shared__ cplx urow[2][LU_NB];  // pivot row of column c, for the bulk wavefronts
  __shared__ int s_ready, s_bulk;  // last released pivot; bulk completions

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = (int)blockIdx.x;
  const int rec = jb + 1;
  const int rstr = rec;
  const int cstride = P * rec + jb;
  const __amdgpu_buffer_rsrc_t rs = rec_rsrc(slots);
  // element of the header of workgroup t for column cc
  auto hdr_el = [&](int cc, int t) __attribute__((always_inline)) {
    return SLOT_HDR + cc * P + t;
  };
  const long r0 = (long)j + (long)g * RPW;  // first row of the workgroup
  const int nv = (N - r0 >= RPW) ? RPW : ((N - r0 > 0) ? (int)(N - r0) : 0);
  bool ok = true;

  if constexpr (FUSE) {
    static_assert(RPL == 1, "the fused update holds U12 beside a 64-row panel");
    static_assert(sizeof(T) == sizeof(cplx), "the fused update is built for the FP64 factorisation");
    constexpr int UOFF = LU_NB * (64 + 1);  // U12 in LDS after the panel block
    cplx *Ls = pan;                         // L11, then this workgroup's rows of L21 (ld 64)
    cplx *Us = pan + UOFF;                  // all of U12 (ld 64)
    __shared__ int s_src[64], s_srcx[64];   // row sources of rows r0 + i and j0 + i
    if (tid < 64) {
      s_src[tid] = (int)r0 + tid;
      s_srcx[tid] = j0 + tid;
    }
    __syncthreads();
    {
      const int np = swp0[0];
      for (int e = tid; e < np; e += SNT) {
        const int dst = swp0[1 + 2 * e], src = swp0[2 + 2 * e];
        if (dst >= r0 && dst < r0 + 64) s_src[dst - r0] = src;
        if (dst >= j0 && dst < j0 + 64) s_srcx[dst - j0] = src;
      }
    }
    // L11 of the previous panel into LDS; each wavefront's column of U12 (its
    // interchanged rows j0 .. j0 + 63) into registers
    for (int idx = tid; idx < LU_NB * LU_NB; idx += SNT) {
      const int r = idx & 63, c = idx >> 6;
      st_st(Ls, idx, ld_z(A, (long)(j0 + r) + (long)(j0 + c) * lda));
    }
    __syncthreads();
    const int cown = g + P * wave;  // this wavefront's column of U12
    if (wave < SNT / 64 && cown < jb) {
      const st_v2 x0 = ld_z(A, (long)s_srcx[lane] + (long)(j + cown) * lda);
      cplx x = cmk(x0.x, x0.y);
      for (int c0 = 0; c0 < LU_NB - 1; c0 += 8) {
        cplx lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + u;
          lv[u] = (c < LU_NB - 1 && lane > c) ? Ls[c * 64 + lane] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + u;
          if (c < LU_NB - 1) x = cfms(x, lv[u], readlane_c(x, c));
        }
      }
      rec_store(rs, SLOT_U12 + cown * 64 + lane, x);
    }
    // (columns c = g + P w, w < 7 wavefronts: all of jb <= 64 are covered when P >= 10)
    __syncthreads();  // every wavefront done with L11
    // all of U12 (every load in flight, then polled until written), and this
    // workgroup's rows of L21, into LDS
    {
      constexpr int UPT = (LU_NB * LU_NB + SNT - 1) / SNT;
      bm_v4i uv[UPT];
#pragma unroll
      for (int q = 0; q < UPT; ++q) {
        const int idx = tid + SNT * q;
        if (idx < LU_NB * jb) uv[q] = rec_load(rs, SLOT_U12 + idx);
      }
#pragma unroll
      for (int q = 0; q < UPT; ++q) {
        const int idx = tid + SNT * q;
        if (idx < LU_NB * LU_NB) {
          const int r = idx & 63, kc = idx >> 6;  // L21: row r, column kc of the previous panel
          st_st(Ls, kc * 64 + r, (r < nv) ? ld_z(A, (r0 + r) + (long)(j0 + kc) * lda) : st_v2{0.0, 0.0});
        }
      }
      const unsigned long long t0 = wall_clock64();
      for (;;) {
        bool all = true;
#pragma unroll
        for (int q = 0; q < UPT; ++q) {
          const int idx = tid + SNT * q;
          if (idx < LU_NB * jb && rec_empty(uv[q])) {
            all = false;
            uv[q] = rec_load(rs, SLOT_U12 + idx);
          }
        }
        if (all) break;
        if (!ok || wait_expired(t0)) {
          if (ok) atomicOr(dev_err, 1);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
#pragma unroll
      for (int q = 0; q < UPT; ++q) {
        const int idx = tid + SNT * q;
        if (idx < LU_NB * LU_NB) Us[idx] = (idx < LU_NB * jb) ? rec_value(uv[q]) : cmk(0.0, 0.0);
      }
    }
    __syncthreads();
    // this workgroup's rows: (row sigma(r) of these columns) - L21 U12; wavefronts
    // 0 .. 3 each own a 32 x 32 quarter (2 x 2 blocks of 16 x 16 MFMA results:
    // lane l, register q -> row l % 16, column 4 q + l / 16 of a block)
    pdbl4 accr[2][2], acci[2][2];
    const int wm = wave & 1, wn = (wave >> 1) & 1, fq = lane >> 4, fi = lane & 15;
    if (wave < 4) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accr[a][b] = (pdbl4){0, 0, 0, 0};
          acci[a][b] = (pdbl4){0, 0, 0, 0};
        }
      for (int k4 = 0; k4 < LU_NB; k4 += 4) {
        cplx av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = Ls[(k4 + fq) * 64 + wm * 32 + a * 16 + fi];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Us[(wn * 32 + b * 16 + fi) * 64 + k4 + fq];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            accr[a][b] = pmfma16(bv[b].x, av[a].x, accr[a][b]);
            acci[a][b] = pmfma16(bv[b].y, av[a].x, acci[a][b]);
            accr[a][b] = pmfma16(bv[b].y, -av[a].y, accr[a][b]);
            acci[a][b] = pmfma16(bv[b].x, av[a].y, acci[a][b]);
          }
      }
    }
    __syncthreads();  // L21 read by every wavefront before the panel block overwrites it
    if (wave < 4) {
      st_v2 old[2][2][4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = wm * 32 + a * 16 + fi, c = wn * 32 + b * 16 + 4 * q + fq;
            old[a][b][q] = ld_z(A, (r < nv && c < jb) ? (long)s_src[r] + (long)(j + c) * lda : (long)j + (long)j * lda);
          }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = wm * 32 + a * 16 + fi, c = wn * 32 + b * 16 + 4 * q + fq;
            if (c < jb)
              st_st(pan, c * LDP + r,
                    (r < nv) ? st_v2{old[a][b][q].x - accr[a][b][q], old[a][b][q].y - acci[a][b][q]} : st_v2{0.0, 0.0});
          }
    }
  } else {
    // the workgroup's block of the panel into LDS: each thread's loads in one
    // batch (unconditional, an item outside the block reads the panel's first
    // element), then the LDS stores
    constexpr int PT = (RPW * LU_NB + SNT - 1) / SNT;
    const long a0 = (long)j + (long)j * lda;
    st_v2 v[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int idx = tid + SNT * q, r = idx % RPW, c = idx / RPW;
      v[q] = ld_z(A, (r < nv && c < jb) ? (r0 + r) + (long)(j + c) * lda : a0);
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int idx = tid + SNT * q, r = idx % RPW, c = idx / RPW;
      if (c < jb) st_st(pan, c * LDP + r, (r < nv) ? v[q] : st_v2{0.0, 0.0});
    }
  }
  if (tid == 0) {
    s_ready = -1;
    s_bulk = 0;
  }
  __syncthreads();

  if (wave == 0) {
    const bool col_ok = lane < jb;
    // candidate among the rows > after of a column held as x[k] = row lane + 64 k:
    // (value, local row), wave-uniform; ties go to the smallest row
    auto cand = [&](const cplx(&x)[RPL], long after, double &vmax, int &lr) __attribute__((always_inline)) {
      double v[RPL], best = -1.0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        v[k] = (r < nv && r0 + r > after) ? l1abs(x[k]) : -1.0;
        best = fmax(best, v[k]);
      }
      vmax = wave_max_f64(best);
      lr = -1;
      if (vmax >= 0.0) {
#pragma unroll
        for (int k = RPL - 1; k >= 0; --k) {
          const unsigned long long m = __ballot(v[k] == vmax);
          if (m) lr = 64 * k + (int)__ffsll((long long)m) - 1;
        }
      }
    };
    // records of column cc: the header (value, row) as soon as the candidate is known
    auto publish_head = [&](int cc, double v, int lr) __attribute__((always_inline)) {
      if (lane == 0) rec_store(rs, hdr_el(cc, g), (lr >= 0) ? cmk(v, (double)(r0 + lr)) : cmk(-1.0, -1.0));
    };
    // then (for column 0) the candidate row lr and the diagonal row; columns > cc
    // still owe the update of pivot cc - 1 (multipliers in column cc - 1, pivot row pr)
    auto publish_rows = [&](int cc, int lr, cplx pr) __attribute__((always_inline)) {
      const int base = cc * cstride;
      const int sc = base + g * rstr;
      const bool late = (cc > 0) && lane > cc;
      const long ld = (long)j + cc - r0;
      const bool has_d = (ld >= 0 && ld < nv);
      cplx x = cmk(0, 0), y = cmk(0, 0);
      if (col_ok && lr >= 0) {
        x = pan[lane * LDP + lr];
        if (late) x = cfms(x, pan[(cc - 1) * LDP + lr], pr);
      }
      if (col_ok && has_d) {
        y = pan[lane * LDP + (int)ld];
        if (late) y = cfms(y, pan[(cc - 1) * LDP + (int)ld], pr);
      }
      if (col_ok) rec_store(rs, sc + 1 + lane, x);  // zeros when the workgroup has no candidate
      if (col_ok && has_d) rec_store(rs, base + P * rstr + lane, y);
    };
    cplx xc[RPL], xn[RPL];  // columns c and c + 1 of the workgroup's rows
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      xc[k] = pan[lane + 64 * k];
      xn[k] = (jb > 1) ? pan[LDP + lane + 64 * k] : cmk(0, 0);
    }
    {
      double v;
      int lr;
      cand(xc, (long)j - 1, v, lr);
      publish_head(0, v, lr);
      publish_rows(0, lr, cmk(0, 0));
    }
    // interchange bookkeeping (workgroup 0): lane l holds the source row of panel
    // position j + l, and of the l-th further row touched by the interchanges
    int pcont = j + lane, epos = -1, econt = 0, nextra = 0;

    for (int c = 0; c < jb; ++c) {
      const long gc = (long)j + c;
      const int base = c * cstride;
      // receive the headers (lanes < P)
      bm_v4i vh;
      const int eh = (lane < P) ? hdr_el(c, lane) : -1;
      if (eh >= 0) vh = rec_load(rs, eh);
      {
        const unsigned long long t0 = wall_clock64();
        for (;;) {
          const bool all = eh < 0 || !rec_empty(vh);
          if (__all(all)) break;
          if (!all) vh = rec_load(rs, eh);
          if (!ok || wait_expired(t0)) {
            if (ok) atomicOr(dev_err, 1);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      // winner: largest value, then the smallest workgroup index (= smallest row)
      double vw = -1.0;
      long pw = -1;
      int ww = -1;
      if (P <= 64) {
        const cplx h = (eh >= 0) ? rec_value(vh) : cmk(-1.0, -1.0);
        double vm;
        const int fl = wave_argmax_first(h.x, vm);
        if (fl >= 0) {
          ww = fl;
          vw = vm;
          pw = (long)readlane_f64(h.y, fl);
        }
      } else {
        // more than 64 workgroups: the headers again through the record buffer
        double lv = -1.0;
        for (int t = lane; t < P; t += 64) lv = fmax(lv, rec_poll(rs, hdr_el(c, t), dev_err, ok).x);
        lv = wave_max_f64(lv);
        int li = 0x7fffffff;
        if (lv >= 0.0)
          for (int t = lane; t < P; t += 64)
            if (rec_poll(rs, hdr_el(c, t), dev_err, ok).x == lv) {
              li = t;
              break;
            }
        li = wave_min_int(li);
        if (li != 0x7fffffff) {
          ww = li;
          vw = lv;
          pw = (long)rec_poll(rs, hdr_el(c, li), dev_err, ok).y;
        }
      }
      if (ww < 0) {  // no comparable candidate (a column of NaNs): keep the diagonal row, report it
        vw = 0.0;
        pw = gc;
      }
      const long p = pw;
      // the winner's row and the diagonal row, both loads in flight together
      cplx dr = cmk(0, 0), pr;
      {
        const int ed = col_ok ? base + P * rstr + lane : -1;
        const int er = (col_ok && ww >= 0) ? base + ww * rstr + 1 + lane : -1;
        bm_v4i vd, vr;
        if (ed >= 0) vd = rec_load(rs, ed);
        if (er >= 0) vr = rec_load(rs, er);
        const unsigned long long t0 = wall_clock64();
        for (;;) {
          const bool okd = ed < 0 || !rec_empty(vd), okr = er < 0 || !rec_empty(vr);
          if (__all(okd && okr)) break;
          if (!okd) vd = rec_load(rs, ed);
          if (!okr) vr = rec_load(rs, er);
          if (!ok || wait_expired(t0)) {
            if (ok) atomicOr(dev_err, 1);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (ed >= 0) dr = rec_value(vd);
        pr = (er >= 0) ? rec_value(vr) : dr;
      }
      // row interchange (row gc <- pivot row, row p <- old row gc), multipliers of
      // column c and the update of column c + 1 (held in registers since the last
      // step), in registers only: the candidate's header for column c + 1 goes out
      // before any LDS access
      const long lg = gc - r0, lp = p - r0;
      const bool have_next = (c + 1 < jb), have_next2 = (c + 2 < jb);
      const cplx pc = readlane_c(pr, c), dcv = readlane_c(dr, c);
      const cplx u1 = readlane_c(pr, have_next ? c + 1 : c), d1 = readlane_c(dr, have_next ? c + 1 : c);
      cplx x1[RPL], lv[RPL];
#pragma unroll
      for (int k = 0; k < RPL; ++k) x1[k] = xn[k];
      if (p != gc) {
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int r = lane + 64 * k;
          xc[k] = csel(r == (int)lg, pc, xc[k]);
          xc[k] = csel(r == (int)lp, dcv, xc[k]);
          x1[k] = csel(r == (int)lg, u1, x1[k]);
          x1[k] = csel(r == (int)lp, d1, x1[k]);
        }
      }
      const cplx ip = (vw == 0.0) ? cmk(0, 0) : pivot_recip(pc);
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        lv[k] = cmul(xc[k], ip);
        if (r < nv && r0 + r > gc) x1[k] = cfms(x1[k], lv[k], u1);
      }
      double v = -1.0;
      int lr = -1;
      if (have_next) {
        cand(x1, gc, v, lr);
        publish_head(c + 1, v, lr);
      }
      // the bulk wavefronts must have finished the previous pivot (columns >= c + 2)
      if (c >= 1 && c - 1 <= jb - 3) {
        const unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(&s_bulk, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < SNB * c) {
          if (!ok || wait_expired(t0)) {
            if (ok) atomicOr(dev_err, 1);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      // the record rows of column c + 1 (candidate row lr, diagonal row gc + 1) from
      // the registers and the LDS as it stands before this step's writes: row lp
      // already counts as holding the old row gc (dr); column c is the multiplier, column
      // c + 1 the updated value, columns > c + 1 still owe pivot c
      if (have_next) {
        auto rec_row = [&](int r) __attribute__((always_inline)) -> cplx {
          cplx lr_c = cmk(0, 0), x1_c = cmk(0, 0);
#pragma unroll
          for (int k = 0; k < RPL; ++k)
            if ((r >> 6) == k) {
              lr_c = readlane_c(lv[k], r & 63);
              x1_c = readlane_c(x1[k], r & 63);
            }
          cplx b = (r == (int)lp) ? dr : pan[lane * LDP + r];
          if (lane == c) b = lr_c;
          else if (lane == c + 1) b = x1_c;
          else if (lane > c + 1) b = cfms(b, lr_c, pr);
          return b;
        };
        const int base1 = (c + 1) * cstride;
        const long ld = gc + 1 - r0;
        const bool has_d = (ld >= 0 && ld < nv);
        if (col_ok) rec_store(rs, base1 + g * rstr + 1 + lane, (lr >= 0) ? rec_row(lr) : cmk(0, 0));
        if (col_ok && has_d) rec_store(rs, base1 + P * rstr + lane, rec_row((int)ld));
      }
      // now LDS: the interchanged rows; column c + 2 with pivot c applied, kept in
      // registers for the next step (in LDS it stays one pivot behind, like the
      // columns the bulk wavefronts update); the multipliers; column c + 1 from the
      // pivot row down (the pivot row's entry is final); the pivot row
      if (p != gc && col_ok) {
        if (lg >= 0 && lg < nv) pan[lane * LDP + (int)lg] = pr;
        if (lp >= 0 && lp < nv) pan[lane * LDP + (int)lp] = dr;
      }
      const cplx u2 = readlane_c(pr, have_next2 ? c + 2 : c);
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        cplx x2 = have_next2 ? pan[(c + 2) * LDP + r] : cmk(0, 0);
        if (r < nv && r0 + r > gc) x2 = cfms(x2, lv[k], u2);
        xn[k] = x2;
      }
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        if (r < nv && r0 + r >= gc) {
          if (r0 + r > gc) pan[c * LDP + r] = lv[k];
          if (have_next) pan[(c + 1) * LDP + r] = x1[k];
        }
      }
      if (col_ok) urow[c & 1][lane] = pr;
      // release pivot c to the bulk wavefronts
      if (lane == 0) __hip_atomic_store(&s_ready, c, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
      for (int k = 0; k < RPL; ++k) xc[k] = x1[k];
      if (g == 0) {
        if (lane == 0) {
          ipiv[gc] = (int32_t)p;
          if (vw == 0.0 && dev_err[1] == 0) dev_err[1] = (int32_t)(gc + 1);
        }
        const int ca = __builtin_amdgcn_readlane(pcont, c);
        const bool inpanel = p < (long)j + jb;
        int cb, eidx = -1;
        if (inpanel) {
          cb = __builtin_amdgcn_readlane(pcont, (int)(p - j));
        } else {
          const unsigned long long mk = __ballot(lane < nextra && epos == (int)p);
          if (mk) {
            eidx = (int)__ffsll((long long)mk) - 1;
            cb = __builtin_amdgcn_readlane(econt, eidx);
          } else {
            eidx = nextra++;
            cb = (int)p;
            if (lane == eidx) epos = (int)p;
          }
        }
        pcont = (lane == c) ? cb : pcont;
        pcont = (inpanel && lane == (int)(p - j)) ? ca : pcont;
        econt = (!inpanel && lane == eidx) ? ca : econt;
      }
    }
    // net permutation of the panel's interchanges on rows >= j: pairs (dst, src)
    if (g == 0) {
      const bool m1 = col_ok && pcont != j + lane;
      const bool m2 = lane < nextra && econt != epos;
      const unsigned long long b1 = __ballot(m1), b2 = __ballot(m2);
      const int n1 = __popcll(b1);
      const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      if (m1) {
        const int k = __popcll(b1 & below);
        swp[1 + 2 * k] = j + lane;
        swp[2 + 2 * k] = pcont;
      }
      if (m2) {
        const int k = n1 + __popcll(b2 & below);
        swp[1 + 2 * k] = epos;
        swp[2 + 2 * k] = econt;
      }
      if (lane == 0) swp[0] = n1 + __popcll(b2);
    }
  } else {
    // bulk wavefronts: pivot c's update of columns >= c + 3, one step behind; the
    // loads of a batch of BU columns are issued before any store
    constexpr int NG = (SNB * 64) / RPW;  // column groups
    constexpr int BU = 4;
    const int bt = tid - 64;
    const int r = bt % RPW, grp = bt / RPW;
    for (int c = 0; c + 2 < jb; ++c) {
      {
        const unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(&s_ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < c) {
          if (!ok || wait_expired(t0)) {
            if (ok) atomicOr(dev_err, 1);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (grp < NG && r < nv && r0 + r > (long)j + c) {
        const cplx l = pan[c * LDP + r];
        for (int cc0 = c + 3 + grp; cc0 < jb; cc0 += NG * BU) {
          cplx av[BU], uv[BU];
#pragma unroll
          for (int b = 0; b < BU; ++b) {
            const int cc = cc0 + b * NG;
            if (cc < jb) {
              av[b] = pan[cc * LDP + r];
              uv[b] = urow[c & 1][cc];
            }
          }
#pragma unroll
          for (int b = 0; b < BU; ++b) {
            const int cc = cc0 + b * NG;
            if (cc < jb) pan[cc * LDP + r] = cfms(av[b], l, uv[b]);
          }
        }
      }
      if (lane == 0) __hip_atomic_fetch_add(&s_bulk, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();

  for (int idx = tid; idx < RPW * jb; idx += SNT) {
    const int r = idx % RPW, c = idx / RPW;
    if (r < nv) st_z(A, (r0 + r) + (long)(j + c) * lda, to_v2(pan[c * LDP + r]));
  }
  // refill the words the next panel uses in the other slot buffer with the empty pattern
  if (next_P > 0) {
    const int nrec = next_jb + 1, nrstr = nrec;
    const int ncstr = next_P * nrec + next_jb;
    const int per_col = next_P * nrec + next_jb;
    unsigned long long *ns = (unsigned long long *)next_slots;
    for (int idx = g * SNT + tid; idx < next_jb * per_col; idx += P * SNT) {
      const int col = idx / per_col, rem = idx % per_col;
      const int el = col * ncstr + ((rem < next_P * nrec) ? (rem / nrec) * nrstr + rem % nrec
                                                           : next_P * nrstr + (rem - next_P * nrec));
      ns[2 * (size_t)el] = SENT;
      ns[2 * (size_t)el + 1] = SENT;
    }
    for (int idx = g * SNT + tid; idx < 2 * next_jb * next_P; idx += P * SNT) ns[2 * (size_t)SLOT_HDR + idx] = SENT;
    for (int idx = g * SNT + tid; idx < 2 * LU_NB * LU_NB; idx += P * SNT) ns[2 * (size_t)SLOT_U12 + idx] = SENT;
  }
  if constexpr (FUSE) {
    // U12: rows j0 .. j0 + 63 of this panel's columns
    if (g == 0) {
      const cplx *Us = pan + LU_NB * (64 + 1);
      for (int idx = tid; idx < LU_NB * jb; idx += SNT) {
        const int k = idx & 63, cc = idx >> 6;
        st_z(A, (long)(j0 + k) + (long)(j + cc) * lda, to_v2(Us[cc * 64 + k]));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 2. row interchanges outside the panel, and U12 = L11^{-1} A12
//
// Workgroups [0, nleft): SWAP_COLS columns each of [0, lcols), interchanges only.
// Workgroups [nleft, ...): CW columns each of [c0, c1): interchanges, then
// forward substitution with the unit lower L11 (in LDS) on rows j .. j + jb - 1,
// lane = row, CW / 4 columns per wavefront, the solved value of row c broadcast
// from lane c by readlane.  The substitution is a chain of jb - 1 dependent steps
// whose length is set by the instructions each SIMD issues per step, so the launch
// on the path to the next panel takes one column per wavefront (CW = 4) and the
// launches beside the next panel two (CW = 8, half the workgroups).
// The kernel sits on the path from one panel to the next, so its global loads are
// issued in batches (each thread's loads of a phase are in flight together):
// the interchange pairs with L11 and the block rows, then the interchange
// sources.  Work items are mapped by fixed strides (64 rows, 2 LU_NB pairs), with
// no division; every load is issued unconditionally (an item outside the block
// reads the block's first element) so that no branch separates the loads, and
// only the stores are predicated.
// ---------------------------------------------------------------------------
#define BM_LU_EVENT_FLAGS hipEventDisableSystemFence
#define SWAP_COLS 16
#define ST_CW_NEXT 4  // columns per workgroup, next panel's columns
#define ST_CW_REST 8  // columns per workgroup, the other columns
#define ST_NPAIR (2 * LU_NB)  // at most 2 jb rows change place
#define ST_LDS(cw) ((size_t)(LU_NB * LU_NB + (cw) * LU_NB) * sizeof(cplx))

template <int CW, class T, bool BAT = false>
__global__ __launch_bounds__(256) void swap_trsm_kernel(T *A, long lda, int j, int jb, int lcols, int c0, int c1,
                                                        const int32_t *swp, int nleft, bm_lu_batch bb) {
  if constexpr (BAT) {
    A = (T *)bb.A[blockIdx.y];
    swp = bb.swp[blockIdx.y];
  }
  extern __shared__ cplx sm[];
  __shared__ int s_pair[2 * ST_NPAIR];  // (dst, src) rows of the interchange
  const int np = swp[0];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nleft) {
    if (np == 0) return;
    if (tid < 2 * np) s_pair[tid] = swp[1 + tid];
    __syncthreads();
    constexpr int LPT = ST_NPAIR * SWAP_COLS / 256;
    const int cbase = blockIdx.x * SWAP_COLS;
    st_v2 v[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = tid + 256 * q, e = idx % ST_NPAIR, col = cbase + idx / ST_NPAIR;
      const bool ok = e < np && col < lcols;
      v[q] = ld_z(A, ok ? s_pair[2 * e + 1] + (long)col * lda : (long)j);
    }
    __syncthreads();  // every source read before any row is overwritten
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = tid + 256 * q, e = idx % ST_NPAIR, col = cbase + idx / ST_NPAIR;
      if (e < np && col < lcols) st_z(A, s_pair[2 * e] + (long)col * lda, v[q]);
    }
    return;
  }
  static_assert(CW % 4 == 0 && CW * LU_NB % 256 == 0 && ST_NPAIR * CW % 256 == 0, "column split");
  constexpr int CPW = CW / 4;  // columns per wavefront
  const int cw0 = c0 + ((int)blockIdx.x - nleft) * CW;
  const int ncw = (c1 - cw0 < CW) ? c1 - cw0 : CW;
  cplx *Ls = sm;                 // L11, column-major, ld LU_NB
  cplx *X = Ls + LU_NB * LU_NB;  // rows j .. j + jb - 1 of the columns, [CW][LU_NB]
  constexpr int LPT_L = LU_NB * LU_NB / 256, LPT_X = CW * LU_NB / 256, LPT_S = ST_NPAIR * CW / 256;
  // phase 1: the pairs, L11 and the block rows, all in flight together
  const long a0 = (long)j + (long)j * lda;  // L11's first element: the address of items outside the block
  const int pr_v = swp[1 + ((tid < 2 * np) ? tid : 0)];
  st_v2 lv[LPT_L], xv[LPT_X];
#pragma unroll
  for (int q = 0; q < LPT_L; ++q) {
    const int idx = tid + 256 * q, r = idx % LU_NB, c = idx / LU_NB;
    lv[q] = ld_z(A, (r < jb && c < jb) ? (j + r) + (long)(j + c) * lda : a0);
  }
#pragma unroll
  for (int q = 0; q < LPT_X; ++q) {
    const int idx = tid + 256 * q, r = idx % LU_NB, cl = idx / LU_NB;
    xv[q] = ld_z(A, (r < jb && cl < ncw) ? (j + r) + (long)(cw0 + cl) * lda : a0);
  }
  if (tid < 2 * np) s_pair[tid] = pr_v;
  __syncthreads();
  // phase 2: the interchange sources
  st_v2 sv[LPT_S];
#pragma unroll
  for (int q = 0; q < LPT_S; ++q) {
    const int idx = tid + 256 * q, e = idx % ST_NPAIR, cl = idx / ST_NPAIR;
    sv[q] = ld_z(A, (e < np && cl < ncw) ? s_pair[2 * e + 1] + (long)(cw0 + cl) * lda : a0);
  }
#pragma unroll
  for (int q = 0; q < LPT_L; ++q) {
    const int idx = tid + 256 * q, r = idx % LU_NB, c = idx / LU_NB;
    if (r < jb && c < jb) st_st(Ls, c * LU_NB + r, lv[q]);
  }
#pragma unroll
  for (int q = 0; q < LPT_X; ++q) {
    const int idx = tid + 256 * q, r = idx % LU_NB, cl = idx / LU_NB;
    if (r < jb && cl < ncw) st_st(X, cl * LU_NB + r, xv[q]);
  }
  __syncthreads();  // every source read (and X filled) before any destination is written
#pragma unroll
  for (int q = 0; q < LPT_S; ++q) {
    const int idx = tid + 256 * q, e = idx % ST_NPAIR, cl = idx / ST_NPAIR;
    if (e < np && cl < ncw) {
      const int dst = s_pair[2 * e];
      if (dst < j + jb) st_st(X, cl * LU_NB + (dst - j), sv[q]);
      else st_z(A, dst + (long)(cw0 + cl) * lda, sv[q]);
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const bool row_ok = lane < jb;
  cplx xs[CPW];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int cl = CPW * wave + q;
    xs[q] = (row_ok && cl < ncw) ? X[cl * LU_NB + lane] : cmk(0, 0);
  }
  // the multipliers of eight steps are read from LDS ahead of them, so that a step's
  // chain is only the broadcast of row c and one complex multiply-add
  for (int c0 = 0; c0 < jb - 1; c0 += 8) {
    st_v2 lvv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      const st_v2 z = {0.0, 0.0};
      const st_v2 t = *reinterpret_cast<const st_v2 *>(Ls + (c < LU_NB ? c : LU_NB - 1) * LU_NB + lane);
      lvv[u] = (c < jb - 1 && lane > c && row_ok) ? t : z;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      if (c < jb - 1) {
        const cplx l = cmk(lvv[u].x, lvv[u].y);
#pragma unroll
        for (int q = 0; q < CPW; ++q) xs[q] = cfms(xs[q], l, readlane_c(xs[q], c));
      }
    }
  }
  if (row_ok) {
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int cl = CPW * wave + q;
      if (cl < ncw) st_z(A, (j + lane) + (long)(cw0 + cl) * lda, to_v2(xs[q]));
    }
  }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------

struct bm_lu_pipe;
static void pipe_destroy(bm_lu_pipe *q);

bm_getrf_ws *bm_getrf_ws_create(int n) {
  bm_getrf_ws *w = new bm_getrf_ws();
  w->n = n;
  w->npanel = (n + LU_NB - 1) / LU_NB;
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  bool ok = hipMalloc(&w->slots, sizeof(cplx) * 2 * SLOT_ELEMS) == hipSuccess;
  ok = ok && hipMalloc(&w->swp, sizeof(int32_t) * (size_t)w->npanel * SWP_STRIDE) == hipSuccess;
  ok = ok && hipMalloc(&w->zbuf, sizeof(cplx) * (1 + 2 * (size_t)nblk * BM_DIAG_NB * BM_MAX_NRHS)) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking) == hipSuccess;
  // the lookahead events only order the two streams of this device: no system-scope
  // fence (the host never inspects them)
  ok = ok && hipEventCreateWithFlags(&w->e_next, hipEventDisableTiming | BM_LU_EVENT_FLAGS) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&w->e_rest, hipEventDisableTiming | BM_LU_EVENT_FLAGS) == hipSuccess;
  if (!ok) {
    bm_getrf_ws_destroy(w);
    return nullptr;
  }
  return w;
}

void bm_getrf_ws_destroy(bm_getrf_ws *w) {
  if (!w) return;
  (void)hipFree(w->slots);
  (void)hipFree(w->swp);
  (void)hipFree(w->zbuf);
  if (w->aux) {
    (void)hipStreamSynchronize(w->aux);
    (void)hipStreamDestroy(w->aux);
  }
  if (w->e_next) (void)hipEventDestroy(w->e_next);
  if (w->e_rest) (void)hipEventDestroy(w->e_rest);
  pipe_destroy(w->pipe);
  delete w;
}

template <class TS>
__global__ void diag_inv_kernel(int n, const TS *LU, long ld, cplx *dinv);

#define TI_LDS ((size_t)(2 * TI_N * (TI_N + 1) + 1024) * sizeof(cplx))  // M, X, T of tri_inv64

template <class T>
using panel_fn = void (*)(int, T *, long, int, int, int, int32_t *, int32_t *, cplx *, cplx *, int, int, int32_t *,
                          int, const int32_t *, bm_lu_batch);
// 64 and 128 rows per workgroup; 64 rows with the previous panel's update fused
// (FP64 storage only)
static const panel_fn<cplx> panel_fns[3] = {panel_kernel<1, false, cplx>, panel_kernel<2, false, cplx>,
                                            panel_kernel<1, true, cplx>};
static const panel_fn<cplx32> panel_fns_c64[2] = {panel_kernel<1, false, cplx32>, panel_kernel<2, false, cplx32>};
static const panel_fn<cplx> panel_fns_bat[2] = {panel_kernel<1, false, cplx, true>, panel_kernel<2, false, cplx, true>};
static const panel_fn<cplx32> panel_fns_bat_c64[2] = {panel_kernel<1, false, cplx32, true>,
                                                      panel_kernel<2, false, cplx32, true>};
static const void *panel_bat_of(const cplx *, int k) { return (const void *)panel_fns_bat[k]; }
static const void *panel_bat_of(const cplx32 *, int k) { return (const void *)panel_fns_bat_c64[k]; }
static const void *panel_fn_of(const cplx *, int k) { return (const void *)panel_fns[k]; }
static const void *panel_fn_of(const cplx32 *, int k) { return (k < 2) ? (const void *)panel_fns_c64[k] : nullptr; }

static int panel_attr_done[64];

// Fill of 8-byte words (the error flags and the exchange sentinels).  A kernel
// rather than hipMemsetAsync so that the factorisation can be captured in a HIP
// graph and replayed.
__global__ void fill_u64_kernel(unsigned long long *p, size_t n, unsigned long long v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

int bm_fill_u64(hipStream_t s, void *p, size_t n, unsigned long long v) {
  if (n == 0) return BM_OK;
  size_t nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)nb), dim3(256), 0, s, (unsigned long long *)p, n, v);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// rows per lane of the chain wavefront (1: 64, 2: 128 rows per workgroup) and the
// workgroup count of a panel of R rows: 64 rows per workgroup while that keeps
// P <= PANEL_RPL1_PMAX, else 128
static bool panel_shape(int R, int ncu, int *rpl, int *P_out) {
  const int pmax = (ncu < PANEL_PMAX) ? ncu : PANEL_PMAX;
  int k = (R <= 64 * PANEL_RPL1_PMAX) ? 1 : 2;
  const int P = (R + 64 * k - 1) / (64 * k);
  if (P < 1 || P > pmax) return false;
  *rpl = k;
  *P_out = P;
  return true;
}

size_t bm_getrf_ws_bytes(int n) {
  const size_t npanel = (size_t)(n + LU_NB - 1) / LU_NB, nblk = (size_t)(n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  return sizeof(cplx) * 2 * SLOT_ELEMS + sizeof(int32_t) * npanel * SWP_STRIDE +
         sizeof(cplx) * (1 + 2 * nblk * BM_DIAG_NB * BM_MAX_NRHS);
}

// Dynamic-LDS limits of the factorisation kernels on the current device (once per
// device; called before any stream capture of the factorisation).
int bm_getrf_prepare() {
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !panel_attr_done[dev]) {
    const void *big[] = {(const void *)panel_fns[0],     (const void *)panel_fns[1],
                         (const void *)panel_fns[2],     (const void *)panel_fns_c64[0],
                         (const void *)panel_fns_c64[1], (const void *)panel_fns_bat[0],
                         (const void *)panel_fns_bat[1], (const void *)panel_fns_bat_c64[0],
                         (const void *)panel_fns_bat_c64[1]};
    for (const void *f : big)
      BM_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PANEL_LDS_ALLOC));
    const void *st_next[] = {(const void *)swap_trsm_kernel<ST_CW_NEXT, cplx>,
                             (const void *)swap_trsm_kernel<ST_CW_NEXT, cplx32>,
                             (const void *)swap_trsm_kernel<ST_CW_NEXT, cplx, true>,
                             (const void *)swap_trsm_kernel<ST_CW_NEXT, cplx32, true>};
    const void *st_rest[] = {(const void *)swap_trsm_kernel<ST_CW_REST, cplx>,
                             (const void *)swap_trsm_kernel<ST_CW_REST, cplx32>,
                             (const void *)swap_trsm_kernel<ST_CW_REST, cplx, true>,
                             (const void *)swap_trsm_kernel<ST_CW_REST, cplx32, true>};
    for (int t = 0; t < 4; ++t) {
      BM_HIP_TRY(hipFuncSetAttribute(st_next[t], hipFuncAttributeMaxDynamicSharedMemorySize, (int)ST_LDS(ST_CW_NEXT)));
      BM_HIP_TRY(hipFuncSetAttribute(st_rest[t], hipFuncAttributeMaxDynamicSharedMemorySize, (int)ST_LDS(ST_CW_REST)));
    }
    BM_HIP_TRY(hipFuncSetAttribute((const void *)diag_inv_kernel<cplx>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)TI_LDS));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)diag_inv_kernel<cplx32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)TI_LDS));
    panel_attr_done[dev] = 1;
  }
  return BM_OK;
}

// The k = 64 update C -= L21 U12 of an LU step: FP64 storage on the FP64 matrix
// cores or, with gemm32, beyond the next panel on the FP32 ones; complex64 storage
// on the FP64 shallow kernel for the next panel, on the FP32 matrix cores beyond.
static int lu_gemm(hipStream_t st, int m, int n, int k, const cplx *A, long lda, const cplx *B, long ldb, cplx *C,
                   long ldc, bool next, int gemm32) {
  const cplx one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  return ((gemm32 && !next) ? bm_launch_zgemm32 : bm_launch_zgemm)(st, m, n, k, mone, A, lda, B, ldb, one, C, ldc);
}
static int lu_gemm(hipStream_t st, int m, int n, int k, const cplx32 *A, long lda, const cplx32 *B, long ldb,
                   cplx32 *C, long ldc, bool next, int) {
  const cplx one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  return (next ? bm_launch_zgemm_shallow_c64 : bm_launch_zgemm32_cc)(st, m, n, k, mone, A, lda, B, ldb, one, C, ldc);
}

// The interchanges of the panel at column j (jb columns, list swp) on the columns
// [0, lcols), and on the columns [c0, c1) right of it also U12 = L11^{-1} A12 and
// the trailing update A22 -= L21 U12 (FP32 matrix cores with gemm32).  `next`:
// the narrow column split for the next panel's columns (critical path).
template <class T>
static int lu_update(hipStream_t st, T *A, long lda, int n, int j, int jb, const int32_t *swp, int lcols, int c0,
                     int c1, bool next, int gemm32) {
  const int cw = next ? ST_CW_NEXT : ST_CW_REST;
  const int nleft = (lcols + SWAP_COLS - 1) / SWAP_COLS, nright = (c1 > c0) ? (c1 - c0 + cw - 1) / cw : 0;
  if (nleft + nright > 0) {
    if (next)
      hipLaunchKernelGGL((swap_trsm_kernel<ST_CW_NEXT, T>), dim3(nleft + nright), dim3(256), ST_LDS(ST_CW_NEXT), st, A,
                         lda, j, jb, lcols, c0, c1, swp, nleft, bm_lu_batch{});
    else
      hipLaunchKernelGGL((swap_trsm_kernel<ST_CW_REST, T>), dim3(nleft + nright), dim3(256), ST_LDS(ST_CW_REST), st, A,
                         lda, j, jb, lcols, c0, c1, swp, nleft, bm_lu_batch{});
    BM_HIP_TRY(hipGetLastError());
  }
  const int nr = n - j - jb, jn = j + jb;
  if (nr > 0 && c1 > c0)
    // gemm32: the FP32 matrix cores for the columns beyond the next panel (the
    // next panel's 64 columns, on the critical path, keep the FP64 shallow kernel)
    return lu_gemm(st, nr, c1 - c0, jb, A + jn + (long)j * lda, lda, A + j + (long)c0 * lda, lda,
                   A + jn + (long)c0 * lda, lda, next, gemm32);
  return BM_OK;
}

// Common start of a factorisation: panel shapes (rows per lane, workgroups) and
// the device flags and the first panel's exchange words reset.
static int lu_begin(hipStream_t s, int n, int32_t *dev_err, bm_getrf_ws *w, int *shape, int *ncu_out) {
  if (int rc0 = bm_getrf_prepare()) return rc0;
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  int ncu = 0;
  BM_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  *ncu_out = ncu;
  if (int rc0 = bm_fill_u64(s, dev_err, 1, 0ull)) return rc0;  // [0] error, [1] info
  const int npanel = (n + LU_NB - 1) / LU_NB;
  if (npanel > 1024) return BM_E_ARG;
  for (int pi = 0; pi < npanel; ++pi) {
    const int R = n - pi * LU_NB;
    if (!panel_shape(R, ncu, &shape[3 * pi], &shape[3 * pi + 1])) return BM_E_ARG;
  }
  if (npanel > 0) {  // the first panel's words of slot buffer 0; each panel refills the next one's
    const int jb0 = (n < LU_NB) ? n : LU_NB;
    const size_t cstr0 = (size_t)shape[1] * (jb0 + 1) + jb0;
    if (int rc0 = bm_fill_u64(s, w->slots, 2 * (size_t)jb0 * cstr0, ~0ull)) return rc0;
    if (int rc0 = bm_fill_u64(s, w->slots + SLOT_HDR, 2 * (size_t)jb0 * shape[1], ~0ull)) return rc0;
  }
  return BM_OK;
}

// Launch of panel pi (all P workgroups must run at the same time: P <= the CU
// count, checked in panel_shape, and one workgroup fits a CU, so on a device that
// is not saturated by other work every workgroup is resident at once; a plain
// launch avoids the start and drain cost of a cooperative launch.  Every wait in
// the kernel is bounded, so a launch whose workgroups cannot all become resident
// ends with BM_E_DEVICE, not a hang.)
// whether panel pi applies the previous panel's update to its own columns itself
// (64 rows per workgroup, enough workgroups to solve U12 one column per wavefront).
// Only in the factorisation beside the Schur product, where the two separate
// launches it replaces wait for CUs held by the product's other work; alone on
// the device they are as fast (measured: the plain 4096 x 4096 LU 11.05 ms with
// them, 11.15 ms fused; star2048 beside the product 6.86 ms per step with them,
// 6.79 ms fused).
static bool lu_fused(bool overlap, const int *shape, int pi) {
  return overlap && pi >= 1 && shape[3 * pi] == 1 && shape[3 * pi + 1] >= 10;
}

template <class T>
static int lu_panel(hipStream_t s, int n, T *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w,
                    const int *shape, int pi, bool overlap) {
  const int npanel = (n + LU_NB - 1) / LU_NB;
  const int j = pi * LU_NB, jb = (n - j < LU_NB) ? n - j : LU_NB;
  int P = shape[3 * pi + 1];
  int next_P = 0, next_jb = 0;
  if (pi + 1 < npanel) {
    next_jb = (n - j - LU_NB < LU_NB) ? n - j - LU_NB : LU_NB;
    next_P = shape[3 * (pi + 1) + 1];
  }
  cplx *cur = w->slots + (size_t)(pi & 1) * SLOT_ELEMS, *nxt = w->slots + (size_t)((pi + 1) & 1) * SLOT_ELEMS;
  int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
  long ldal = (long)lda;
  int nn = n, jj = j, jbb = jb;
  const bool fuse = lu_fused(overlap, shape, pi);
  int j0 = fuse ? j - LU_NB : 0;
  const int32_t *swp0 = fuse ? w->swp + (size_t)(pi - 1) * SWP_STRIDE : swp;
  bm_lu_batch bb{};
  void *args[] = {&nn, &A, &ldal, &jj, &jbb, &P, &ipiv, &dev_err, &cur, &nxt, &next_P, &next_jb, &swp, &j0, &swp0, &bb};
  const int rpl = shape[3 * pi];
  if (w->prof) bm_phase_begin(w->prof, BM_PH_PANEL);
  BM_HIP_TRY(hipLaunchKernel(panel_fn_of(A, fuse ? 2 : rpl - 1), dim3(P), dim3(SNT), args, PANEL_LDS_ALLOC, s));
  if (w->prof) bm_phase_end(w->prof, BM_PH_PANEL);
  return BM_OK;
}

template <class T>
static int getrf_run(hipStream_t s, int n, T *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w,
                     int gemm32) {
  if (!w || w->n < n) return BM_E_ARG;
  int shape[3 * 1024];  // rows per lane, P per panel
  int ncu = 0;
  if (int rc0 = lu_begin(s, n, dev_err, w, shape, &ncu)) return rc0;
  const int npanel = (n + LU_NB - 1) / LU_NB;
  // (a workspace without the second stream runs every update on s, in order)
  const bool la = w->aux != nullptr;
  for (int j = 0, pi = 0; j < n; j += LU_NB, ++pi) {
    const int jb = (n - j < LU_NB) ? n - j : LU_NB;
    if (int rc = lu_panel(s, n, A, lda, ipiv, dev_err, w, shape, pi, false)) return rc;
    const int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
    // Lookahead: the stream s applies the panel's interchanges and its update to the
    // next panel's columns only; the auxiliary stream applies them to every other
    // column while s factors the next panel.  s waits for that rest of panel k - 1
    // before it touches the columns of panel k + 1 (which were part of it).
    const int nr = n - j - jb;
    const int jn = j + jb, jbn = (nr < LU_NB) ? nr : LU_NB;  // next panel's columns [jn, jn + jbn)
    if (la && pi > 0) BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
    int rc = lu_update(s, A, (long)lda, n, j, jb, swp, 0, jn, jn + jbn, true, gemm32);
    if (rc) return rc;
    if (la) {
      BM_HIP_TRY(hipEventRecord(w->e_next, s));
      BM_HIP_TRY(hipStreamWaitEvent(w->aux, w->e_next, 0));
    }
    rc = lu_update(la ? w->aux : s, A, (long)lda, n, j, jb, swp, j, jn + jbn, n, false, gemm32);
    if (rc) return rc;
    if (la) BM_HIP_TRY(hipEventRecord(w->e_rest, w->aux));
  }
  if (w->aux && npanel > 0) BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
  return BM_OK;
}

int bm_getrf_run(hipStream_t s, int n, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w,
                 int gemm32) {
  return getrf_run(s, n, A, lda, ipiv, dev_err, w, gemm32);
}

int bm_getrf_run_c64(hipStream_t s, int n, cplx32 *A, int64_t lda, int32_t *ipiv, int32_t *dev_err,
                     bm_getrf_ws *w) {
  return getrf_run(s, n, A, lda, ipiv, dev_err, w, 1);
}

// ---------------------------------------------------------------------------
// The LU of a batch of problems of one order: the single-problem sequence (panel,
// the next panel's update on s, the other columns' update on the second stream),
// each launch covering every problem (blockIdx.y), so that the CUs one problem's
// panel chain leaves idle work on the others.  Every problem sees the kernels and
// the arithmetic of its own factorisation (bitwise the same factors).
// ---------------------------------------------------------------------------
static int lu_gemm_batch(const cplx *, hipStream_t st, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                         long lda, long ob, long oc, bool) {
  return bm_launch_zgemm_lu_batch(st, count, bb, m, n, k, oa, lda, ob, lda, oc, lda);
}
static int lu_gemm_batch(const cplx32 *, hipStream_t st, int count, const bm_lu_batch &bb, int m, int n, int k,
                         long oa, long lda, long ob, long oc, bool next) {
  return (next ? bm_launch_zgemm_shallow_lu_batch_c64 : bm_launch_zgemm32_lu_batch)(st, count, bb, m, n, k, oa, lda, ob,
                                                                                    lda, oc, lda);
}

template <class T>
static int lu_update_batch(hipStream_t st, int count, const bm_lu_batch &bb, long lda, int n, int j, int jb,
                           int lcols, int c0, int c1, bool next) {
  const int cw = next ? ST_CW_NEXT : ST_CW_REST;
  const int nleft = (lcols + SWAP_COLS - 1) / SWAP_COLS, nright = (c1 > c0) ? (c1 - c0 + cw - 1) / cw : 0;
  if (nleft + nright > 0) {
    const dim3 grid(nleft + nright, count);
    if (next)
      hipLaunchKernelGGL((swap_trsm_kernel<ST_CW_NEXT, T, true>), grid, dim3(256), ST_LDS(ST_CW_NEXT), st,
                         (T *)nullptr, lda, j, jb, lcols, c0, c1, (const int32_t *)nullptr, nleft, bb);
    else
      hipLaunchKernelGGL((swap_trsm_kernel<ST_CW_REST, T, true>), grid, dim3(256), ST_LDS(ST_CW_REST), st,
                         (T *)nullptr, lda, j, jb, lcols, c0, c1, (const int32_t *)nullptr, nleft, bb);
    BM_HIP_TRY(hipGetLastError());
  }
  const int nr = n - j - jb, jn = j + jb;
  if (nr > 0 && c1 > c0)
    return lu_gemm_batch((const T *)nullptr, st, count, bb, nr, c1 - c0, jb, jn + (long)j * lda, lda,
                         j + (long)c0 * lda, jn + (long)c0 * lda, next);
  return BM_OK;
}

template <class T>
static int getrf_run_batch(hipStream_t s, int n, int count, T *const *A, int64_t lda, int32_t *const *ipiv,
                           int32_t *const *dev_err, bm_getrf_ws *const *ws) {
  if (count < 1 || count > BM_LU_BATCH_MAX || n < 1 || lda < n) return BM_E_ARG;
  for (int b = 0; b < count; ++b)
    if (!ws[b] || ws[b]->n < n || !A[b] || !ipiv[b] || !dev_err[b]) return BM_E_ARG;
  int shape[3 * 1024];
  int ncu = 0;
  for (int b = 0; b < count; ++b)  // per problem: flags and the first panel's exchange words
    if (int rc0 = lu_begin(s, n, dev_err[b], ws[b], shape, &ncu)) return rc0;
  // every workgroup of a batched panel must be resident at once
  if ((long)count * shape[1] > ncu) return BM_E_ARG;
  bm_getrf_ws *w = ws[0];
  const bool la = w->aux != nullptr;
  bm_lu_batch bb{};
  for (int b = 0; b < count; ++b) {
    bb.A[b] = (cplx *)A[b];  // (complex64 storage read back as such by the T kernels)
    bb.ipiv[b] = ipiv[b];
    bb.err[b] = dev_err[b];
  }
  const long ldal = (long)lda;
  const int npanel = (n + LU_NB - 1) / LU_NB;
  for (int j = 0, pi = 0; j < n; j += LU_NB, ++pi) {
    const int jb = (n - j < LU_NB) ? n - j : LU_NB;
    int P = shape[3 * pi + 1], next_P = 0, next_jb = 0;
    if (pi + 1 < npanel) {
      next_jb = (n - j - LU_NB < LU_NB) ? n - j - LU_NB : LU_NB;
      next_P = shape[3 * (pi + 1) + 1];
    }
    for (int b = 0; b < count; ++b) {
      bb.cur[b] = ws[b]->slots + (size_t)(pi & 1) * SLOT_ELEMS;
      bb.nxt[b] = ws[b]->slots + (size_t)((pi + 1) & 1) * SLOT_ELEMS;
      bb.swp[b] = ws[b]->swp + (size_t)pi * SWP_STRIDE;
    }
    {
      int nn = n, jj = j, jbb = jb, j0 = 0;
      T *a0 = nullptr;
      cplx *c0p = nullptr, *c1p = nullptr;
      int32_t *p0 = nullptr, *e0 = nullptr, *s0 = nullptr;
      const int32_t *sw0 = nullptr;
      void *args[] = {&nn, &a0, (void *)&ldal, &jj, &jbb, &P, &p0, &e0, &c0p, &c1p, &next_P, &next_jb, &s0, &j0,
                      &sw0, &bb};
      BM_HIP_TRY(hipLaunchKernel(panel_bat_of((const T *)nullptr, shape[3 * pi] - 1), dim3(P, count), dim3(SNT), args,
                                 PANEL_LDS_ALLOC, s));
    }
    const int nr = n - j - jb;
    const int jn = j + jb, jbn = (nr < LU_NB) ? nr : LU_NB;
    if (la && pi > 0) BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
    if (int rc = lu_update_batch<T>(s, count, bb, ldal, n, j, jb, 0, jn, jn + jbn, true)) return rc;
    if (la) {
      BM_HIP_TRY(hipEventRecord(w->e_next, s));
      BM_HIP_TRY(hipStreamWaitEvent(w->aux, w->e_next, 0));
    }
    if (int rc = lu_update_batch<T>(la ? w->aux : s, count, bb, ldal, n, j, jb, j, jn + jbn, n, false)) return rc;
    if (la) BM_HIP_TRY(hipEventRecord(w->e_rest, w->aux));
  }
  if (la && npanel > 0) BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
  return BM_OK;
}

int bm_getrf_run_batch(hipStream_t s, int n, int count, cplx *const *A, int64_t lda, int32_t *const *ipiv,
                       int32_t *const *dev_err, bm_getrf_ws *const *ws) {
  return getrf_run_batch(s, n, count, A, lda, ipiv, dev_err, ws);
}

int bm_getrf_run_batch_c64(hipStream_t s, int n, int count, cplx32 *const *A, int64_t lda, int32_t *const *ipiv,
                           int32_t *const *dev_err, bm_getrf_ws *const *ws) {
  return getrf_run_batch(s, n, count, A, lda, ipiv, dev_err, ws);
}

// ---------------------------------------------------------------------------
// LU of A = alpha Bot Top with the product computed beside the panels
// (the Schur complement of Theorem thm:LU; FP64)
//
// The product is formed in column segments of whole 64-column blocks.  Block 0
// goes first on the whole device (k split into slices summed afterwards, so that
// its few tiles fill the CUs); the other segments follow on a third stream g as a
// bounded persistent grid of one workgroup per CU that claims each of its CUs
// whole, leaving free as many CUs as the largest panel has workgroups plus
// SP_FREE_CUS for the updates, while the panels factor the columns that are
// already there.  A segment whose first panel is f is brought up to date by a
// fourth stream c: the interchanges, U12 rows and trailing updates of panels
// 0 .. f - 2 on its columns, in panel order, each as soon as its panel is done;
// from panel f - 1 on the segment belongs to the ordinary lookahead (s for the
// next panel's columns, aux for the others).  The catch-up reads every panel's L
// columns as the panel left them, so the interchanges of later panels on the
// columns left of them are deferred to c, after the last catch-up.
//
// The segment widths come from a timing model of the device (one 64 x 64 tile of
// depth k on a CU that holds one workgroup: 0.12 us per unit of k; a panel of the
// chain: 0.15 ms; a catch-up step: 12 us plus its GEMM at 25 TFLOP/s): each
// segment is the widest whose product and catch-up end before the panels reach
// it, so that the chain never waits; a wrong model costs time, never correctness.
// ---------------------------------------------------------------------------
#define SP_MAXB (BM_PIPE_MAX_N / LU_NB)
#define SP_MAXSEG 24
#define SP_FREE_CUS 32

struct bm_lu_pipe {
  hipStream_t g, c;
  hipEvent_t e_in, e_cdone, ep[SP_MAXB], es[SP_MAXSEG], ec[SP_MAXSEG];
};

static void pipe_destroy(bm_lu_pipe *q) {
  if (!q) return;
  if (q->g) {
    (void)hipStreamSynchronize(q->g);
    (void)hipStreamDestroy(q->g);
  }
  if (q->c) {
    (void)hipStreamSynchronize(q->c);
    (void)hipStreamDestroy(q->c);
  }
  hipEvent_t *evs[] = {&q->e_in, &q->e_cdone};
  for (hipEvent_t *e : evs)
    if (*e) (void)hipEventDestroy(*e);
  for (int i = 0; i < SP_MAXB; ++i)
    if (q->ep[i]) (void)hipEventDestroy(q->ep[i]);
  for (int i = 0; i < SP_MAXSEG; ++i) {
    if (q->es[i]) (void)hipEventDestroy(q->es[i]);
    if (q->ec[i]) (void)hipEventDestroy(q->ec[i]);
  }
  delete q;
}

int bm_getrf_pipe_create(bm_getrf_ws *w) {
  if (!w) return BM_E_ARG;
  if (w->pipe) return BM_OK;
  bm_lu_pipe *q = new (std::nothrow) bm_lu_pipe();
  if (!q) return BM_E_NOMEM;
  memset((void *)q, 0, sizeof(*q));
  const unsigned fl = hipEventDisableTiming | BM_LU_EVENT_FLAGS;
  bool ok = hipStreamCreateWithFlags(&q->g, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&q->c, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&q->e_in, fl) == hipSuccess &&
            hipEventCreateWithFlags(&q->e_cdone, fl) == hipSuccess;
  for (int i = 0; ok && i < SP_MAXB; ++i) ok = hipEventCreateWithFlags(&q->ep[i], fl) == hipSuccess;
  for (int i = 0; ok && i < SP_MAXSEG; ++i)
    ok = hipEventCreateWithFlags(&q->es[i], fl) == hipSuccess && hipEventCreateWithFlags(&q->ec[i], fl) == hipSuccess;
  if (!ok) {
    pipe_destroy(q);
    return BM_E_HIP;
  }
  w->pipe = q;
  return BM_OK;
}

size_t bm_getrf_pipe_w_elems(int n) {
  // split-K partials: block 0 over the whole device (at most 16 slices of n x 64)
  // or one round of the bounded grid (at most 256 tiles of 64 x 64)
  const size_t a = (size_t)16 * n * LU_NB, b = (size_t)256 * 64 * 64;
  return a > b ? a : b;
}

struct sp_seg {
  int b0, b1, ks;  // blocks [b0, b1), k split into ks slices
};

// k-slices of a product of `tiles` tiles on `slots` workgroups: enough to fill
// them in one round, at most 16, each at least 256 deep (the three-multiplication
// form), and the partials within the workspace
static int sp_ksplit(int tiles, int slots, int k, size_t w_cap) {
  int ks = (tiles <= slots) ? slots / tiles : 1;
  const int kmax = (k / 256 > 1) ? k / 256 : 1;
  if (ks > kmax) ks = kmax;
  if (ks > 16) ks = 16;
  while (ks > 1 && (size_t)ks * tiles * 64 * 64 > w_cap) --ks;
  return ks < 1 ? 1 : ks;
}

static double sp_time(int tiles, int ks, int slots, int k, double per_k) {
  int kc = (k + ks - 1) / ks;
  kc = (kc + 15) / 16 * 16;
  const int rounds = (tiles * ks + slots - 1) / slots;
  return rounds * per_k * kc + (ks > 1 ? 0.006 : 0.0);
}

// Returns 1 when the planned product ends before the chain of panels (the overlap
// pays), else 0 (then the product is better formed in full first).
static int sp_plan(int n, int k, int ncu, int gs, size_t w_cap, sp_seg *seg, int *nseg_out) {
  const int B = (n + LU_NB - 1) / LU_NB, tb = B;  // blocks; row tiles of a block
  const double per_k1 = 0.49 / 4096.0;            // ms per unit of k: one workgroup per CU
  const double per_k2 = 0.84 / 4096.0;            // two per CU (block 0, whole device)
  const double beta = 0.15 + 0.05 * ((n > 2048) ? (n - 2048) / 2048.0 : 0.0), margin = 0.03;
  int nseg = 0;
  const int ks0 = sp_ksplit(tb, 2 * ncu, k, w_cap);
  const double t0 = sp_time(tb, ks0, 2 * ncu, k, per_k2);
  seg[nseg++] = {0, 1, ks0};
  double E = t0;
  int f = 1;
  while (f < B) {
    int best = 1, bks = sp_ksplit(tb, gs, k, w_cap);
    double bt = sp_time(tb, bks, gs, k, per_k1);
    for (int b = 2; b <= B - f; ++b) {
      const int ks = sp_ksplit(tb * b, gs, k, w_cap);
      const double t = sp_time(tb * b, ks, gs, k, per_k1), fin = E + t;
      int a = (int)((fin - t0) / beta);
      if (a > f - 1) a = f - 1;
      if (a < 0) a = 0;
      const double step = 0.012 + 8.0 * n * (64.0 * b) * 64.0 / 25e9;
      if (fin + a * step <= t0 + beta * f - margin) {
        best = b;
        bks = ks;
        bt = t;
      }
    }
    // the last segment takes the rest; so does a segment that would leave a single
    // block, which alone would need a catch-up step for every panel before it
    if (nseg == SP_MAXSEG - 1 || (B - f - best == 1 && nseg >= 2)) {
      best = B - f;
      bks = sp_ksplit(tb * best, gs, k, w_cap);
      bt = sp_time(tb * best, bks, gs, k, per_k1);
    }
    seg[nseg++] = {f, f + best, bks};
    E += bt;
    f += best;
  }
  *nseg_out = nseg;
  return (E <= t0 + beta * B - margin) ? 1 : 0;
}

int bm_getrf_schur_run(hipStream_t s, int n, cplx alpha, const cplx *bot, int64_t ldbot, const cplx *top,
                       int64_t ldtop, int k, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w,
                       cplx *W, size_t w_elems, int *nseg_out) {
  if (!w || w->n < n || n < 1 || n > BM_PIPE_MAX_N || !w->aux || !w->pipe || k < 1 || !W || !nseg_out ||
      w_elems < bm_getrf_pipe_w_elems(n))
    return BM_E_ARG;
  *nseg_out = 0;
  bm_lu_pipe *q = w->pipe;
  int shape[3 * SP_MAXB];
  int ncu = 0;
  if (int rc0 = lu_begin(s, n, dev_err, w, shape, &ncu)) return rc0;
  const int B = (n + LU_NB - 1) / LU_NB;
  int pmax = 0;
  for (int pi = 0; pi < B; ++pi) pmax = (shape[3 * pi + 1] > pmax) ? shape[3 * pi + 1] : pmax;
  // the product's workgroups: one per CU, leaving free the largest panel's CUs and
  // SP_FREE_CUS more for the trailing updates and catch-ups (which share no CU
  // with the product)
  int gs = ncu - pmax - SP_FREE_CUS;
  if (gs < (ncu - pmax) / 2) gs = ncu - pmax;
  if (gs < 1) return BM_E_ARG;
  sp_seg seg[SP_MAXSEG];
  int nseg = 0;
  bm_problem *ps = w->prof_schur;
  if (!sp_plan(n, k, ncu, gs, w_elems, seg, &nseg)) {
    // the product would not keep ahead of the panels: form it in full first
    if (ps) bm_phase_begin_on(ps, BM_PH_SCHUR, s);
    if (int rc0 = bm_launch_zgemm(s, n, n, k, alpha, bot, ldbot, top, ldtop, cmk(0.0, 0.0), A, lda)) return rc0;
    if (ps) bm_phase_end_on(ps, BM_PH_SCHUR, s);
    return bm_getrf_run(s, n, A, lda, ipiv, dev_err, w, 0);
  }
  *nseg_out = nseg;
  const long ldal = (long)lda;
  auto cols = [&](int i, int *c0, int *c1) {
    *c0 = seg[i].b0 * LU_NB;
    *c1 = (seg[i].b1 * LU_NB < n) ? seg[i].b1 * LU_NB : n;
  };
  // block 0 over the whole device, then the other segments on g (the product's
  // span, from block 0's start on s to the last segment's end on g, is timed)
  if (ps) bm_phase_begin_on(ps, BM_PH_SCHUR, s);
  {
    int c0, c1;
    cols(0, &c0, &c1);
    if (int rc0 = bm_launch_zgemm_persist(s, n, c1 - c0, k, alpha, bot, ldbot, top, ldtop, A, lda, 2 * ncu,
                                          seg[0].ks, W, w_elems, 0))
      return rc0;
  }
  BM_HIP_TRY(hipEventRecord(q->e_in, s));
  BM_HIP_TRY(hipStreamWaitEvent(q->g, q->e_in, 0));
  for (int i = 1; i < nseg; ++i) {
    int c0, c1;
    cols(i, &c0, &c1);
    if (int rc0 = bm_launch_zgemm_persist(q->g, n, c1 - c0, k, alpha, bot, ldbot, top + (long)c0 * ldtop, ldtop,
                                          A + (long)c0 * lda, lda, gs, seg[i].ks, W, w_elems, 1))
      return rc0;
    BM_HIP_TRY(hipEventRecord(q->es[i], q->g));
  }
  if (ps) bm_phase_end_on(ps, BM_PH_SCHUR, nseg > 1 ? q->g : s);
  // the catch-up stream's work, in order: per segment its product, the updates of
  // panels 0 .. f - 2, its completion event; then the deferred left interchanges
  // of panels 1 .. B - 1.  Items are issued once their panel has been issued.
  struct item {
    int type, i, p;  // 0: wait for segment i's product, 1: catch-up step, 2: record, 3: left interchanges
  };
  item items[SP_MAXSEG * (SP_MAXB + 2) + SP_MAXB];
  int nit = 0;
  for (int i = 1; i < nseg; ++i) {
    items[nit++] = {0, i, -1};
    for (int p = 0; p <= seg[i].b0 - 2; ++p) items[nit++] = {1, i, p};
    items[nit++] = {2, i, -1};
  }
  for (int p = 1; p < B; ++p) items[nit++] = {3, 0, p};
  int next_item = 0;
  auto issue = [&](int h) -> int {
    while (next_item < nit && items[next_item].p <= h) {
      const item it = items[next_item++];
      if (it.type == 0) {
        BM_HIP_TRY(hipStreamWaitEvent(q->c, q->es[it.i], 0));
      } else if (it.type == 2) {
        BM_HIP_TRY(hipEventRecord(q->ec[it.i], q->c));
      } else {
        const int j = it.p * LU_NB, jb = (n - j < LU_NB) ? n - j : LU_NB;
        const int32_t *swp = w->swp + (size_t)it.p * SWP_STRIDE;
        BM_HIP_TRY(hipStreamWaitEvent(q->c, q->ep[it.p], 0));
        if (it.type == 1) {
          int c0, c1;
          cols(it.i, &c0, &c1);
          if (int rc0 = lu_update(q->c, A, ldal, n, j, jb, swp, 0, c0, c1, false, 0)) return rc0;
        } else {
          // the L columns of panels < p are read by the updates of their own
          // panels, the last of which (p - 1, on aux) is behind e_rest
          BM_HIP_TRY(hipStreamWaitEvent(q->c, w->e_rest, 0));
          if (int rc0 = lu_update(q->c, A, ldal, n, j, jb, swp, j, 0, 0, false, 0)) return rc0;
        }
      }
    }
    return BM_OK;
  };
  if (int rc0 = issue(-1)) return rc0;
  for (int pi = 0; pi < B; ++pi) {
    const int j = pi * LU_NB, jb = (n - j < LU_NB) ? n - j : LU_NB;
    if (int rc = lu_panel(s, n, A, lda, ipiv, dev_err, w, shape, pi, true)) return rc;
    BM_HIP_TRY(hipEventRecord(q->ep[pi], s));
    if (int rc = issue(pi)) return rc;
    const int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
    const int nr = n - j - jb;
    const int jn = j + jb, jbn = (nr < LU_NB) ? nr : LU_NB;
    if (pi > 0) BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
    int hi = 0;  // end of the columns that follow the lookahead after this panel
    for (int i = 0; i < nseg; ++i)
      if (seg[i].b0 <= pi + 1) {
        int c0, c1;
        cols(i, &c0, &c1);
        hi = c1;
        if (i > 0 && seg[i].b0 == pi + 1) BM_HIP_TRY(hipStreamWaitEvent(s, q->ec[i], 0));  // joins now
      }
    // (a fused next panel applies this update to its own columns; then nothing runs
    // on s after the panel, and the other stream starts from the panel's own event)
    if (!(pi + 1 < B && lu_fused(true, shape, pi + 1))) {
      if (int rc = lu_update(s, A, ldal, n, j, jb, swp, 0, jn, jn + jbn, true, 0)) return rc;
      BM_HIP_TRY(hipEventRecord(w->e_next, s));
      BM_HIP_TRY(hipStreamWaitEvent(w->aux, w->e_next, 0));
    } else {
      BM_HIP_TRY(hipStreamWaitEvent(w->aux, q->ep[pi], 0));
    }
    for (int i = 1; i < nseg; ++i)
      if (seg[i].b0 == pi + 1) BM_HIP_TRY(hipStreamWaitEvent(w->aux, q->ec[i], 0));
    if (int rc = lu_update(w->aux, A, ldal, n, j, jb, swp, 0, jn + jbn, hi, false, 0)) return rc;
    BM_HIP_TRY(hipEventRecord(w->e_rest, w->aux));
  }
  if (int rc = issue(B)) return rc;
  if (next_item != nit) return BM_E_ARG;  // (every item's panel exists)
  BM_HIP_TRY(hipEventRecord(q->e_cdone, q->c));
  BM_HIP_TRY(hipStreamWaitEvent(s, q->e_cdone, 0));
  BM_HIP_TRY(hipStreamWaitEvent(s, w->e_rest, 0));
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free LU (bm_zgetrf_noalloc): the factorisation's scratch memory (the
// two exchange-slot buffers of the panels, the per-panel interchange lists and the
// two device flags) lives in one file-scope device array instead of memory the
// call allocates.  Host code never uses the array's name as a device address: its
// address on each device comes from hipGetSymbolAddress, taken once per device on
// the first call there.  All calls on one device share the array, so calls that
// overlap in time on one device race; each call refills what must start empty.
// Without the second stream (which would have to be created) every trailing update
// runs on the caller's stream after the next panel's own update.
// ---------------------------------------------------------------------------
#define NA_SLOTS_BYTES (sizeof(cplx) * 2 * SLOT_ELEMS)
#define NA_SWP_BYTES (sizeof(int32_t) * (size_t)(BM_NOALLOC_MAX_N / LU_NB) * SWP_STRIDE)
#define NA_SCRATCH_BYTES (NA_SLOTS_BYTES + NA_SWP_BYTES + 256)
static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

#define NA_MAX_DEV 64
static void *na_ptr[NA_MAX_DEV];
static std::mutex na_mutex;

static int na_scratch(int dev, unsigned char **out) {
  if (dev < 0 || dev >= NA_MAX_DEV) return BM_E_HIP;
  std::lock_guard<std::mutex> lk(na_mutex);
  if (!na_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BM_E_HIP;
    na_ptr[dev] = ptr;
  }
  *out = (unsigned char *)na_ptr[dev];
  return BM_OK;
}

extern "C" int bm_zgetrf_noalloc(void *hip_stream, int32_t n, void *A, int64_t lda, int32_t *ipiv, int32_t *info) {
  if (n < 0 || n > BM_NOALLOC_MAX_N || lda < n || (n > 0 && (!A || !ipiv))) return BM_E_ARG;
  if (n == 0) {
    if (info) *info = 0;
    return BM_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  unsigned char *sp = nullptr;
  if (int rc = na_scratch(dev, &sp)) return rc;
  bm_getrf_ws w{};  // host view of the scratch; no stream, no events, no profiling
  w.n = BM_NOALLOC_MAX_N;
  w.npanel = BM_NOALLOC_MAX_N / LU_NB;
  w.slots = (cplx *)sp;
  w.swp = (int32_t *)(sp + NA_SLOTS_BYTES);
  w.zbuf = nullptr;
  w.aux = nullptr;
  w.e_next = w.e_rest = nullptr;
  int32_t *dev_err = (int32_t *)(sp + NA_SLOTS_BYTES + NA_SWP_BYTES);
  int rc = bm_getrf_run(s, n, (cplx *)A, lda, ipiv, dev_err, &w, 0);
  if (rc || !info) return rc;
  int32_t h[2] = {0, 0};
  BM_HIP_TRY(hipMemcpyAsync(h, dev_err, sizeof(h), hipMemcpyDeviceToHost, s));
  BM_HIP_TRY(hipStreamSynchronize(s));
  *info = h[1];
  return h[0] ? BM_E_DEVICE : BM_OK;
}

// ---------------------------------------------------------------------------
// solve support: inverses of the 64 x 64 diagonal blocks of L (unit lower) and U,
// and each inverse times the off-diagonal block the triangular solve meets last
//   WL_b = Linv_b L(b, b - 1),  WU_b = Uinv_b U(b, b + 1)
// so that the solve of block b can apply its inverse before the block it depends
// on last is known: x_b = inv(D_b) r_b - W_b x_{b -+ 1}, with r_b the right-hand side
// less every other off-diagonal product.
// dinv layout: block b at dinv + b * 4 * 64 * 64: [Linv, Uinv, WL, WU] (col-major 64x64;
// a tile that does not exist, WL_0 or WU_last, is not written)
// ---------------------------------------------------------------------------
template <class TS>
__global__ __launch_bounds__(256) void diag_inv_kernel(int n, const TS *LU, long ld, cplx *dinv) {
  extern __shared__ cplx sm[];
  cplx *Ms = sm, *Xs = sm + TI_N * (TI_N + 1), *T = sm + 2 * TI_N * (TI_N + 1);
  const int b = blockIdx.x;
  const int o = b * BM_DIAG_NB;
  const int nb = (n - o < BM_DIAG_NB) ? n - o : BM_DIAG_NB;
  {
    // the block, every load of a thread in flight together (entries outside a ragged
    // block read its first element and are replaced by the identity's)
    constexpr int LPT = TI_N * TI_N / 256;
    st_v2 v[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % TI_N, c = idx / TI_N;
      v[q] = ld_z(LU, (r < nb && c < nb) ? (o + r) + (long)(o + c) * ld : o + (long)o * ld);
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % TI_N, c = idx / TI_N;
      Ms[r + c * (TI_N + 1)] = (r < nb && c < nb) ? cmk(v[q].x, v[q].y) : cmk(r == c ? 1.0 : 0.0, 0.0);
    }
  }
  __syncthreads();
  // workgroup (b, 0) inverts the unit lower triangle, (b, 1) the upper one
  const int up = blockIdx.y;
  cplx *Xo = dinv + (size_t)b * BM_DINV_TILES * TI_N * TI_N + (size_t)up * TI_N * TI_N;
  if (!up)
    tri_inv64<true>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  else
    tri_inv64<false>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) Xo[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
  // W = inverse times the off-diagonal block: L(b, b - 1) (rows of a ragged last
  // block b beyond n are zero) or U(b, b + 1) (columns beyond n are zero)
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  if (up ? b + 1 >= nblk : b == 0) return;
  const int co = up ? o + BM_DIAG_NB : o - BM_DIAG_NB;
  const int cn = (n - co < BM_DIAG_NB) ? n - co : BM_DIAG_NB;
  {
    constexpr int LPT = TI_N * TI_N / 256;
    st_v2 v[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % TI_N, c = idx / TI_N;
      v[q] = ld_z(LU, (r < nb && c < cn) ? (o + r) + (long)(co + c) * ld : o + (long)co * ld);
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % TI_N, c = idx / TI_N;
      Ms[r + c * (TI_N + 1)] = (r < nb && c < cn) ? cmk(v[q].x, v[q].y) : cmk(0, 0);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, fi = lane & 15, fq = lane >> 4, row = 16 * (threadIdx.x >> 6) + fi;
  st_v2 xt[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const cplx x = Xs[row + (4 * s + fq) * (TI_N + 1)];
    xt[s].x = x.x;
    xt[s].y = x.y;
  }
  cplx *Wo = Xo + 2 * TI_N * TI_N;
#pragma unroll 1
  for (int g = 0; g < TI_N / 8; ++g) {
    double bz[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const cplx m = Ms[(4 * s + fq) + (8 * g + (fi & 7)) * (TI_N + 1)];
      bz[s] = (fi < 8) ? m.x : m.y;
    }
    cplx o0 = cmk(0, 0), o1 = cmk(0, 0);
    tile_mv8(xt, bz, o0, o1, 1.0);
    Wo[row + (8 * g + fq) * TI_N] = o0;
    Wo[row + (8 * g + 4 + fq) * TI_N] = o1;
  }
}

template <class T>
static int diag_inverses(hipStream_t s, int n, const T *LU, int64_t ld, cplx *dinv) {
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  hipLaunchKernelGGL(diag_inv_kernel<T>, dim3(nblk, 2), dim3(256), TI_LDS, s, n, LU, (long)ld, dinv);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_diag_inverses(hipStream_t s, int n, const cplx *LU, int64_t ld, cplx *dinv) {
  return diag_inverses(s, n, LU, ld, dinv);
}

int bm_launch_diag_inverses_c64(hipStream_t s, int n, const cplx32 *LU, int64_t ld, cplx *dinv) {
  return diag_inverses(s, n, LU, ld, dinv);
}

