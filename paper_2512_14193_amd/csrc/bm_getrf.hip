// Blocked right-looking LU with partial pivoting for gfx950 (complex FP64).
//
// Used for U33 = -M31 M13 - M32 M23 (Theorem thm:LU) and, as the comparator, for
// the 2N x 2N ordinary matrix.  Per panel of jb <= 64 columns starting at column j:
//
//  1. panel_kernel (P workgroups of 512 threads, all resident at once): the
//     (n - j) x jb panel lives in registers for the whole panel, one column per lane
//     and RPT consecutive rows per wavefront (workgroups and wavefronts in row
//     order).  In the rank-1 update of column c every row takes its multiplier
//     from lane c by a readlane, so the update touches neither LDS nor memory.  The
//     pivot search of column c + 1 is a scan of lane c + 1 over its rows, then a
//     combine of the eight wavefronts in LDS; each workgroup publishes its candidate
//     (value, row and the whole candidate row) in an exchange record, every
//     workgroup reads all P records, picks the same winner and exchanges the two rows
//     in registers.  One cross-workgroup round trip per column.
//  2. swap_trsm_kernel: the panel's row interchanges, composed into one permutation
//     of at most 2 jb rows, on every column outside the panel; for the columns right
//     of the panel also U12 = L11^{-1} A12 by forward substitution, one wavefront per
//     two columns with lane = row.
//  3. trailing update A22 -= L21 U12 with the MFMA GEMM.
//
// Cross-workgroup data is written with agent-scope stores and read with agent-scope
// loads, which are coherent across the XCDs' separate L2 caches.  Every wait is
// bounded: on expiry the kernel raises the device error flag and runs to completion.
#include "bm_internal.h"
#include "bm_trinv.h"

// ---------------------------------------------------------------------------
// 1. panel factorisation
//
// Exchange protocol: for column c every workgroup g writes one record
//   slots[c][g] = { (value, row), candidate row (jb complex values) }
// and the owner of row j + c also writes that row after the P records.  Slots are filled
// with an all-ones bit pattern before the panel starts (a NaN the arithmetic
// never produces), each 8-byte word is written exactly once with an agent-scope
// store, and readers poll each word with agent-scope loads until it differs from
// the pattern.  So the data itself is the synchronisation: no fence, no counter,
// one round trip per column.  With ONE_ROUND every workgroup receives all P
// records at once; otherwise it receives the P headers and then the winner's row.
// ---------------------------------------------------------------------------
#define PANEL_PMAX 256            // max workgroups of a panel launch
#define PANEL_ONE_ROUND_PMAX 32   // all records of a column are received at once up to this many workgroups
#ifndef PANEL_TARGET_P
#define PANEL_TARGET_P 32         // preferred workgroup count
#endif
#define SENT 0xFFFFFFFFFFFFFFFFULL  // empty exchange word (all ones)
#define PNT 512                   // threads per panel workgroup (8 waves)
#define PNW (PNT / 64)
#define PT_LD 65                  // leading dimension of the LDS transpose tile
#define PANEL_REC_ELEMS (PANEL_ONE_ROUND_PMAX * (LU_NB + 1) > PANEL_PMAX ? PANEL_ONE_ROUND_PMAX * (LU_NB + 1) : PANEL_PMAX)
#define PANEL_LDS_ELEMS (PANEL_REC_ELEMS > LU_NB * PT_LD ? PANEL_REC_ELEMS : LU_NB * PT_LD)
#define PANEL_LDS ((size_t)PANEL_LDS_ELEMS * sizeof(cplx))  // records of a column, or the transpose tile
#define RECV_PT ((PANEL_REC_ELEMS + LU_NB + PNT - 1) / PNT)  // loads per thread per round

// Records of one column sit REC_STRIDE complex values (4 KiB) apart so that the
// reads of a column spread over many memory channels instead of queueing on a few.
#ifndef BM_REC_SPREAD
#define BM_REC_SPREAD 0
#endif
#define REC_STRIDE 256
#define SLOT_ELEMS ((size_t)LU_NB * (PANEL_PMAX + 1) * REC_STRIDE)  // complex values per slot buffer

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

// Panel factorisation, lane = column.  Wavefront w of workgroup g holds RPT
// consecutive rows r0 + w RPT + i (i < RPT) of the panel, lane c holding column c,
// in registers for the whole panel.  Per column c:
//   receive the records of column c; every wavefront selects the same winner p;
//   rows j + c and p exchange (the two wavefronts holding them copy the records);
//   every row below j + c takes its multiplier l = a_c / u_c (computed in lane c,
//   broadcast by readlane) and subtracts l times the pivot row from its columns
//   > c; lane c + 1 scans the updated column for the candidates of column c + 1,
//   the wavefronts combine in LDS and the workgroup publishes its record.
// Exchange layout per column c (rs = record stride, cstride = complex values per column):
//   slots[c * cstride + g * rs]  record of workgroup g: (value, row), then the row
//   slots[c * cstride + P * rs]  the diagonal row j + c, by its owner
// The P workgroups are blockIdx.x = xs g, g = 0 .. P - 1; the launch has xs P
// workgroups and the others return at once (xs = 8 puts all P on one XCD).
template <int RPT, bool ONE_ROUND>
__global__ __launch_bounds__(PNT) void panel_kernel(int N, cplx *A, long lda, int j, int jb, int P, int32_t *ipiv,
                                                    int32_t *dev_err, cplx *slots, cplx *next_slots, int next_P,
                                                    int next_jb, int xs, int32_t *swp) {
  constexpr int RPW = PNW * RPT;           // rows per workgroup
  constexpr int CH = RPW < 64 ? RPW : 64;  // rows per transpose chunk
  extern __shared__ cplx smem[];           // the records of one column, or the transpose tile
  __shared__ cplx drow[LU_NB];
  __shared__ cplx s_cand[PNW];             // per wavefront: (value, local row)

  if ((int)blockIdx.x % xs) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = (int)blockIdx.x / xs;
  const int rec = jb + 1;
  const int rstr = BM_REC_SPREAD ? REC_STRIDE : rec;
  const int cstride = BM_REC_SPREAD ? (P + 1) * REC_STRIDE : P * rec + jb;
  const __amdgpu_buffer_rsrc_t rs = rec_rsrc(slots);
  const long r0 = (long)j + (long)g * RPW;  // first row of the workgroup
  const long wr0 = r0 + (long)wave * RPT;   // first row of the wavefront
  const long wrem = (long)N - wr0;
  const int wn = wrem <= 0 ? 0 : (wrem < RPT ? (int)wrem : RPT);  // rows of the wavefront inside the matrix
  const bool col_ok = lane < jb;
  bool ok = true;
  cplx a[RPT];

  // load: coalesced column reads into the LDS tile, then each wavefront takes its rows
  for (int ch = 0; ch < RPW; ch += CH) {
    for (int idx = tid; idx < CH * jb; idx += PNT) {
      const int r = idx % CH, c = idx / CH;
      const long gr = r0 + ch + r;
      smem[c * PT_LD + r] = (gr < N) ? A[gr + (long)(j + c) * lda] : cmk(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lr = wave * RPT + i - ch;
      if (lr >= 0 && lr < CH) a[i] = csel(col_ok, smem[lane * PT_LD + (lr & (CH - 1))], cmk(0, 0));
    }
    __syncthreads();
  }

  // wavefront candidate of column cc among its rows > after: lane cc scans its rows
  auto wave_candidate = [&](int cc, long after) __attribute__((always_inline)) {
    double best = -1.0;
    int bi = -1;
    if (wr0 > after && wn == RPT) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const double v = l1abs(a[i]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const double v = (i < wn && wr0 + i > after) ? l1abs(a[i]) : -1.0;
        if (v > best) {
          best = v;
          bi = i;
        }
      }
    }
    best = readlane_f64(best, cc);
    bi = __builtin_amdgcn_readlane(bi, cc);
    if (lane == 0) s_cand[wave] = cmk(best, (bi >= 0) ? (double)(wave * RPT + bi) : -1.0);
  };
  // records of column cc: the workgroup's best candidate with its whole row (every
  // record is filled, also without a candidate), and the diagonal row by its owner
  auto publish = [&](int cc) __attribute__((always_inline)) {
    const cplx cw = (lane < PNW) ? s_cand[lane] : cmk(-1.0, -1.0);
    double v;
    const int fw = wave_argmax_first(cw.x, v);  // waves in row order: ties go to the smaller row
    const int lr = (fw >= 0) ? (int)readlane_f64(cw.y, fw) : -1;
    const int base = cc * cstride;
    if (wave == ((lr >= 0) ? lr / RPT : 0)) {
      const int ic = (lr >= 0) ? lr % RPT : -1;
      cplx x = cmk(0, 0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) x = csel(i == ic, a[i], x);
      const int sc = base + g * rstr;
      if (col_ok) rec_store(rs, sc + 1 + lane, x);
      if (lane == 0) rec_store(rs, sc, (lr >= 0) ? cmk(v, (double)(r0 + lr)) : cmk(-1.0, -1.0));
    }
    const long id = (long)j + cc - wr0;
    if (id >= 0 && id < wn) {
      cplx y = cmk(0, 0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) y = csel(i == (int)id, a[i], y);
      if (col_ok) rec_store(rs, base + P * rstr + lane, y);
    }
  };

  wave_candidate(0, (long)j - 1);
  __syncthreads();
  publish(0);

  // interchange bookkeeping (wave 0 of workgroup 0): lane l holds the source row of
  // panel position j + l, and of the l-th further row touched by the interchanges
  int pcont = j + lane, epos = -1, econt = 0, nextra = 0;

  for (int c = 0; c < jb; ++c) {
    const long gc = (long)j + c;
    const int base = c * cstride;
    // receive: every load of the round is issued before any is checked
    {
      const int hdr = ONE_ROUND ? P * rec : P;
      const int total = hdr + jb;
      int ei[RECV_PT];
      bm_v4i v[RECV_PT];
#pragma unroll
      for (int e = 0; e < RECV_PT; ++e) {
        const int idx = tid + PNT * e;
        ei[e] = (idx >= total) ? -1
                : (idx >= hdr) ? base + P * rstr + (idx - hdr)
                : ONE_ROUND    ? base + (idx / rec) * rstr + idx % rec
                               : base + idx * rstr;
        if (ei[e] >= 0) v[e] = rec_load(rs, ei[e]);
      }
      const unsigned long long t0 = wall_clock64();
      for (;;) {
        bool all = true;
#pragma unroll
        for (int e = 0; e < RECV_PT; ++e) {
          if (ei[e] >= 0 && rec_empty(v[e])) {
            all = false;
            v[e] = rec_load(rs, ei[e]);
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
      for (int e = 0; e < RECV_PT; ++e) {
        const int idx = tid + PNT * e;
        if (ei[e] >= 0) {
          if (idx < hdr) smem[idx] = rec_value(v[e]);
          else drow[idx - hdr] = rec_value(v[e]);
        }
      }
    }
    __syncthreads();
    // every wave selects the same winner: largest value, then the smallest
    // workgroup index (= smallest row, the row ranges are in workgroup order)
    double vw = -1.0;
    long pw = -1;
    int ww = -1;
    if (P <= 64) {
      const cplx h = (lane < P) ? (ONE_ROUND ? smem[lane * rec] : smem[lane]) : cmk(-1.0, -1.0);
      double vm;
      const int fl = wave_argmax_first(h.x, vm);
      if (fl >= 0) {
        ww = fl;
        vw = vm;
        pw = (long)readlane_f64(h.y, fl);
      }
    } else {
      double lv = -1.0;
      for (int t = lane; t < P; t += 64) lv = fmax(lv, (ONE_ROUND ? smem[t * rec] : smem[t]).x);
      lv = wave_max_f64(lv);
      int li = 0x7fffffff;
      if (lv >= 0.0)
        for (int t = lane; t < P; t += 64)
          if ((ONE_ROUND ? smem[t * rec] : smem[t]).x == lv) {
            li = t;
            break;
          }
      li = wave_min_int(li);
      if (li != 0x7fffffff) {
        ww = li;
        vw = lv;
        pw = (long)(ONE_ROUND ? smem[li * rec] : smem[li]).y;
      }
    }
    if (ww < 0) {  // no comparable candidate (a column of NaNs): keep the diagonal row, report it
      vw = 0.0;
      pw = gc;
    }
    // pivot row and old diagonal row, one column per lane
    const cplx dr = csel(col_ok, drow[lane], cmk(0, 0));
    cplx pr;
    if (ww < 0) pr = dr;
    else if (ONE_ROUND) pr = csel(col_ok, smem[ww * rec + 1 + lane], cmk(0, 0));
    else pr = col_ok ? rec_poll(rs, base + ww * rstr + 1 + lane, dev_err, ok) : cmk(0, 0);
    const long p = pw;
    if (g == 0 && tid == 0) {
      ipiv[gc] = (int32_t)p;
      if (vw == 0.0 && dev_err[1] == 0) dev_err[1] = (int32_t)(gc + 1);
    }
    // row interchange in registers: row gc <- pivot row, row p <- old row gc
    // (value selects on every slot: a conditional store would index a[] dynamically)
    if (p != gc) {
      const long ia = gc - wr0, ib = p - wr0;
      if (ia >= 0 && ia < RPT) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) a[i] = csel(i == ia, pr, a[i]);
      }
      if (ib >= 0 && ib < RPT) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) a[i] = csel(i == ib, dr, a[i]);
      }
    }
    // multipliers (column c) and the rank-1 update of columns > c, rows > gc: lane c
    // takes l = a_c / u_c, every lane > c subtracts l u (q = u on lanes > c, else 0)
    if (wr0 + wn - 1 > gc) {
      const cplx ip = (vw == 0.0) ? cmk(0, 0) : pivot_recip(readlane_c(pr, c));
      const bool is_c = (lane == c);
      const cplx q = csel(lane > c, pr, cmk(0, 0));
      if (wr0 > gc && wn == RPT) {  // every row of the wavefront is below the pivot
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const cplx t = cmul(a[i], ip);
          const cplx l = readlane_c(t, c);
          a[i] = csel(is_c, t, csub(a[i], cmul(l, q)));
        }
      } else {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const bool upd = i < wn && wr0 + i > gc;
          const cplx t = cmul(a[i], ip);
          const cplx l = csel(upd, readlane_c(t, c), cmk(0, 0));
          a[i] = csel(is_c && upd, t, csub(a[i], cmul(l, q)));
        }
      }
    }
    if (c + 1 < jb) {
      wave_candidate(c + 1, gc);
      __syncthreads();
      publish(c + 1);
    }
    if (g == 0 && wave == 0) {
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
  __syncthreads();

  // write back through the LDS tile (coalesced column writes)
  for (int ch = 0; ch < RPW; ch += CH) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lr = wave * RPT + i - ch;
      if (lr >= 0 && lr < CH && col_ok) smem[lane * PT_LD + lr] = a[i];
    }
    __syncthreads();
    for (int idx = tid; idx < CH * jb; idx += PNT) {
      const int r = idx % CH, c = idx / CH;
      const long gr = r0 + ch + r;
      if (gr < N) A[gr + (long)(j + c) * lda] = smem[c * PT_LD + r];
    }
    __syncthreads();
  }
  // refill the words the next panel uses in the other slot buffer with the empty pattern
  if (next_P > 0) {
    const int nrec = next_jb + 1, nrstr = BM_REC_SPREAD ? REC_STRIDE : nrec;
    const int ncstr = BM_REC_SPREAD ? (next_P + 1) * REC_STRIDE : next_P * nrec + next_jb;
    const int per_col = next_P * nrec + next_jb;
    unsigned long long *ns = (unsigned long long *)next_slots;
    for (int idx = g * PNT + tid; idx < next_jb * per_col; idx += P * PNT) {
      const int col = idx / per_col, rem = idx % per_col;
      const int el = col * ncstr + ((rem < next_P * nrec) ? (rem / nrec) * nrstr + rem % nrec
                                                           : next_P * nrstr + (rem - next_P * nrec));
      ns[2 * (size_t)el] = SENT;
      ns[2 * (size_t)el + 1] = SENT;
    }
  }
  // net permutation of the panel's interchanges on rows >= j: pairs (dst, src)
  if (g == 0 && wave == 0) {
    const bool m1 = lane < jb && pcont != j + lane;
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
}

// ---------------------------------------------------------------------------
// 2. row interchanges outside the panel, and U12 = L11^{-1} A12
//
// Workgroups [0, nleft): SWAP_COLS columns each of [0, j), interchanges only.
// Workgroups [nleft, ...): ST_CW columns each of [j + jb, ncol): interchanges, then
// forward substitution with the unit lower L11 (in LDS) on rows j .. j + jb - 1,
// lane = row, two columns per wavefront, the solved value of row c broadcast from
// lane c by readlane.
// ---------------------------------------------------------------------------
#define SWAP_COLS 16
#define ST_CW 8
#define ST_LDS ((size_t)(LU_NB * LU_NB + ST_CW * LU_NB + 2 * LU_NB * ST_CW) * sizeof(cplx))

__global__ __launch_bounds__(256) void swap_trsm_kernel(cplx *A, long lda, int j, int jb, int ncol, const int32_t *swp,
                                                        int nleft) {
  extern __shared__ cplx sm[];
  const int np = swp[0];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nleft) {
    if (np == 0) return;
    cplx *buf = sm;  // [2 LU_NB][SWAP_COLS]
    const int cbase = blockIdx.x * SWAP_COLS;
    for (int idx = tid; idx < np * SWAP_COLS; idx += 256) {
      const int e = idx % np, col = cbase + idx / np;
      if (col < j) buf[idx] = A[swp[2 + 2 * e] + (long)col * lda];
    }
    __syncthreads();
    for (int idx = tid; idx < np * SWAP_COLS; idx += 256) {
      const int e = idx % np, col = cbase + idx / np;
      if (col < j) A[swp[1 + 2 * e] + (long)col * lda] = buf[idx];
    }
    return;
  }
  const int c0 = j + jb + ((int)blockIdx.x - nleft) * ST_CW;
  const int ncw = (ncol - c0 < ST_CW) ? ncol - c0 : ST_CW;
  cplx *Ls = sm;                     // L11, column-major, ld LU_NB
  cplx *X = Ls + LU_NB * LU_NB;      // rows j .. j + jb - 1 of the columns, [ST_CW][LU_NB]
  cplx *buf = X + ST_CW * LU_NB;     // interchange sources, [2 LU_NB][ST_CW]
  for (int idx = tid; idx < jb * jb; idx += 256) {
    const int r = idx % jb, c = idx / jb;
    Ls[c * LU_NB + r] = A[(j + r) + (long)(j + c) * lda];
  }
  for (int idx = tid; idx < jb * ST_CW; idx += 256) {
    const int r = idx % jb, cl = idx / jb;
    if (cl < ncw) X[cl * LU_NB + r] = A[(j + r) + (long)(c0 + cl) * lda];
  }
  for (int idx = tid; idx < np * ST_CW; idx += 256) {
    const int e = idx % np, cl = idx / np;
    if (cl < ncw) buf[idx] = A[swp[2 + 2 * e] + (long)(c0 + cl) * lda];
  }
  __syncthreads();
  for (int idx = tid; idx < np * ST_CW; idx += 256) {
    const int e = idx % np, cl = idx / np;
    if (cl < ncw) {
      const int dst = swp[1 + 2 * e];
      if (dst < j + jb) X[cl * LU_NB + (dst - j)] = buf[idx];
      else A[dst + (long)(c0 + cl) * lda] = buf[idx];
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int ca = 2 * wave, cb = 2 * wave + 1;
  const bool row_ok = lane < jb;
  cplx xa = (row_ok && ca < ncw) ? X[ca * LU_NB + lane] : cmk(0, 0);
  cplx xb = (row_ok && cb < ncw) ? X[cb * LU_NB + lane] : cmk(0, 0);
  for (int c = 0; c < jb - 1; ++c) {
    const cplx l = (lane > c && row_ok) ? Ls[c * LU_NB + lane] : cmk(0, 0);
    const cplx ya = readlane_c(xa, c), yb = readlane_c(xb, c);
    xa = csub(xa, cmul(l, ya));
    xb = csub(xb, cmul(l, yb));
  }
  if (row_ok) {
    if (ca < ncw) A[(j + lane) + (long)(c0 + ca) * lda] = xa;
    if (cb < ncw) A[(j + lane) + (long)(c0 + cb) * lda] = xb;
  }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------

bm_getrf_ws *bm_getrf_ws_create(int n) {
  bm_getrf_ws *w = new bm_getrf_ws();
  w->n = n;
  w->npanel = (n + LU_NB - 1) / LU_NB;
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  bool ok = hipMalloc(&w->slots, sizeof(cplx) * 2 * SLOT_ELEMS) == hipSuccess;
  ok = ok && hipMalloc(&w->swp, sizeof(int32_t) * (size_t)w->npanel * SWP_STRIDE) == hipSuccess;
  ok = ok && hipMalloc(&w->solve_sync, sizeof(int32_t) * 8) == hipSuccess;
  ok = ok && hipMalloc(&w->zbuf, sizeof(cplx) * (size_t)nblk * BM_DIAG_NB * BM_MAX_NRHS) == hipSuccess;
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
  (void)hipFree(w->solve_sync);
  (void)hipFree(w->zbuf);
  delete w;
}

__global__ void diag_inv_kernel(int n, const cplx *LU, long ld, cplx *dinv);

#define TI_LDS ((size_t)(2 * TI_N * (TI_N + 1) + 1024) * sizeof(cplx))  // M, X, T of tri_inv64

typedef void (*panel_fn)(int, cplx *, long, int, int, int, int32_t *, int32_t *, cplx *, cplx *, int, int, int,
                         int32_t *);
static const panel_fn panel_fns[2][3] = {{panel_kernel<4, false>, panel_kernel<8, false>, panel_kernel<16, false>},
                                         {panel_kernel<4, true>, panel_kernel<8, true>, panel_kernel<16, true>}};

static int panel_attr_done[64];

// rows per wavefront (as an index into {4, 8, 16}: 32, 64 or 128 rows per
// workgroup) and workgroup count of a panel of R rows: the fewest rows per
// wavefront that keep P <= PANEL_TARGET_P, else 16 rows per wavefront and as many
// workgroups as needed
static bool panel_shape(int R, int ncu, int *rpt_idx, int *P_out, int *one_round) {
  const int pmax = (ncu < PANEL_PMAX) ? ncu : PANEL_PMAX;
  int k = 0, P = 0;
  for (k = 0; k < 3; ++k) {
    P = (R + PNW * (4 << k) - 1) / (PNW * (4 << k));
    if (P <= PANEL_TARGET_P) break;
  }
  if (k == 3) k = 2;
  if (P < 1 || P > pmax) return false;
  *rpt_idx = k;
  *P_out = P;
  *one_round = (P <= PANEL_ONE_ROUND_PMAX);
  return true;
}

int bm_getrf_run(hipStream_t s, int n, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w) {
  if (!w || w->n < n) return BM_E_ARG;
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !panel_attr_done[dev]) {
    for (int o = 0; o < 2; ++o)
      for (int k = 0; k < 3; ++k)
        BM_HIP_TRY(hipFuncSetAttribute((const void *)panel_fns[o][k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)PANEL_LDS));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)swap_trsm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)ST_LDS));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)diag_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)TI_LDS));
    panel_attr_done[dev] = 1;
  }
  int ncu = 0;
  BM_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  BM_HIP_TRY(hipMemsetAsync(dev_err, 0, 2 * sizeof(int32_t), s));
  const int npanel = (n + LU_NB - 1) / LU_NB;
  int shape[3 * 1024];  // rows-per-lane index, P, one_round per panel
  if (npanel > 1024) return BM_E_ARG;
  for (int pi = 0; pi < npanel; ++pi) {
    const int R = n - pi * LU_NB;
    if (!panel_shape(R, ncu, &shape[3 * pi], &shape[3 * pi + 1], &shape[3 * pi + 2])) return BM_E_ARG;
  }
  if (npanel > 0) {  // the first panel's words of slot buffer 0; each panel refills the next one's
    const int jb0 = (n < LU_NB) ? n : LU_NB;
    const size_t cstr0 = BM_REC_SPREAD ? (size_t)(shape[1] + 1) * REC_STRIDE : (size_t)shape[1] * (jb0 + 1) + jb0;
    BM_HIP_TRY(hipMemsetAsync(w->slots, 0xFF, sizeof(cplx) * (size_t)jb0 * cstr0, s));
  }
  const cplx one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  for (int j = 0, pi = 0; j < n; j += LU_NB, ++pi) {
    const int jb = (n - j < LU_NB) ? n - j : LU_NB;
    int P = shape[3 * pi + 1];
    int next_P = 0, next_jb = 0;
    if (pi + 1 < npanel) {
      next_jb = (n - j - LU_NB < LU_NB) ? n - j - LU_NB : LU_NB;
      next_P = shape[3 * (pi + 1) + 1];
    }
    // all workgroups of the panel on one XCD (measured slower on MI355X: off)
    int xs = 1;
#ifdef BM_PANEL_XCD
    xs = (BM_PANEL_XCD && ncu >= 256 && P <= ncu / 8) ? 8 : 1;
#endif
    cplx *cur = w->slots + (size_t)(pi & 1) * SLOT_ELEMS, *nxt = w->slots + (size_t)((pi + 1) & 1) * SLOT_ELEMS;
    int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
    long ldal = (long)lda;
    int nn = n, jj = j, jbb = jb;
    void *args[] = {&nn, &A, &ldal, &jj, &jbb, &P, &ipiv, &dev_err, &cur, &nxt, &next_P, &next_jb, &xs, &swp};
    // All P workgroups must run at the same time.  P <= the CU count (checked in
    // panel_shape) and one workgroup fits a CU, so on a device that is not
    // saturated by other work every workgroup is resident at once; a plain launch
    // avoids the start and drain cost of a cooperative launch.  Every wait in the
    // kernel is bounded, so a launch whose workgroups cannot all become resident
    // ends with BM_E_DEVICE, not a hang.
    BM_HIP_TRY(hipLaunchKernel((const void *)panel_fns[shape[3 * pi + 2]][shape[3 * pi]], dim3(xs * P), dim3(PNT),
                               args, PANEL_LDS, s));
    const int nr = n - j - jb;
    const int nleft = (j + SWAP_COLS - 1) / SWAP_COLS, nright = (nr + ST_CW - 1) / ST_CW;
    if (nleft + nright > 0) {
      hipLaunchKernelGGL(swap_trsm_kernel, dim3(nleft + nright), dim3(256), ST_LDS, s, A, ldal, j, jb, n,
                         (const int32_t *)swp, nleft);
      BM_HIP_TRY(hipGetLastError());
    }
    if (nr > 0) {
      const int rc = bm_launch_zgemm(s, nr, nr, jb, mone, A + (j + jb) + (long)j * lda, lda,
                                     A + j + (long)(j + jb) * lda, lda, one, A + (j + jb) + (long)(j + jb) * lda, lda);
      if (rc) return rc;
    }
  }
  return BM_OK;
}

// ---------------------------------------------------------------------------
// solve support: inverses of the 64 x 64 diagonal blocks of L (unit lower) and U
// dinv layout: block b at dinv + b * 2 * 64 * 64: [Linv (col-major 64x64), Uinv]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void diag_inv_kernel(int n, const cplx *LU, long ld, cplx *dinv) {
  extern __shared__ cplx sm[];
  cplx *Ms = sm, *Xs = sm + TI_N * (TI_N + 1), *T = sm + 2 * TI_N * (TI_N + 1);
  const int b = blockIdx.x;
  const int o = b * BM_DIAG_NB;
  const int nb = (n - o < BM_DIAG_NB) ? n - o : BM_DIAG_NB;
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) {
    const int r = idx % TI_N, c = idx / TI_N;
    Ms[r + c * (TI_N + 1)] = (r < nb && c < nb) ? LU[(o + r) + (long)(o + c) * ld] : cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  cplx *Li = dinv + (size_t)b * 2 * TI_N * TI_N, *Ui = Li + TI_N * TI_N;
  tri_inv64<true>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) Li[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
  __syncthreads();
  tri_inv64<false>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) Ui[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
}

int bm_launch_diag_inverses(hipStream_t s, int n, const cplx *LU, int64_t ld, cplx *dinv) {
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3(nblk), dim3(256), TI_LDS, s, n, LU, (long)ld, dinv);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

