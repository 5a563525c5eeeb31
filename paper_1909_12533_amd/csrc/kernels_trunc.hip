// Error-controlled truncation X~ = X + E with ||E|| <= tau (section "Error
// control"), in the Frobenius norm or in the Frob-Inf mixed norm (section
// "Upper bounds for the spectral norm").
//
// Procedure (the paper fixes only the bound): diagonal blocks are never
// removed; the stored off-diagonal upper blocks are grouped in segments
// (Frobenius: one segment, weight 2 for a block and its mirror; Frob-Inf:
// one segment per coarse block (R, S), R <= S, with budget
// (tau / max(m_R, m_S))^2, m_R the number of occupied coarse blocks in coarse
// row R of the full matrix, weight 2 inside diagonal coarse blocks and 1
// elsewhere) and, inside each segment, the longest prefix in ascending
// order of (block norm, block index) is removed whose weighted sum of squared
// norms stays within the budget.
//
// GPU realisation: blocks whose own weighted square already exceeds their
// segment budget can never be removed and are filtered out first (the weights
// are constant inside a segment, so this does not change the prefix); the
// rest is sorted by (segment, norm^2) with a stable LSD radix sort on the
// IEEE bits of norm^2 (monotone for non-negative doubles), so equal norms stay
// in block order; then each segment accumulates its prefix sequentially in
// sorted order and marks removed blocks.  Compaction rewrites only the
// pattern; surviving blocks keep their value slot.
#include "internal.h"

namespace sp2 {

namespace {

constexpr int TPB = 256;
constexpr int RITEMS = 8;
constexpr int RTILE = TPB * RITEMS;
constexpr int RBITS = 4;
constexpr int RDIG = 1 << RBITS;

inline unsigned blocks_for(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_occupancy(const int32_t *row_of, const int32_t *col, int64_t nnzb, int cb, int nc, int32_t *occ) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int R = row_of[b] / cb, S = col[b] / cb;
  occ[R * nc + S] = 1;
  occ[S * nc + R] = 1;
}

// candidate flag: off-diagonal and weight * norm^2 within the segment budget
__global__ void k_cand_flag(const int32_t *row_of, const int32_t *col, int64_t nnzb, const double *nrm2, int cb,
                            int nc, const double *budget, const double *segw, int64_t *flag) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int I = row_of[b], J = col[b];
  int64_t f = 0;
  if (I != J) {
    const int s = (I / cb) * nc + (J / cb);
    f = (segw[s] * nrm2[b] <= budget[s]) ? 1 : 0;
  }
  flag[b] = f;
}

__global__ void k_cand_write(const int32_t *row_of, const int32_t *col, int64_t nnzb, const double *nrm2, int cb,
                             int nc, const int64_t *flag, const int64_t *pos, uint64_t *key, int32_t *seg,
                             int32_t *idx) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb || !flag[b]) return;
  const int64_t o = pos[b];
  key[o] = (uint64_t)__double_as_longlong(nrm2[b]);
  seg[o] = (row_of[b] / cb) * nc + (col[b] / cb);
  idx[o] = (int32_t)b;
}

__global__ void k_bits_range(const uint64_t *key, const int32_t *seg, int64_t n, unsigned long long *kor,
                             unsigned long long *kand, unsigned int *sor, unsigned int *sand) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicOr(kor, (unsigned long long)key[i]);
  atomicAnd(kand, (unsigned long long)key[i]);
  atomicOr(sor, (unsigned int)seg[i]);
  atomicAnd(sand, (unsigned int)seg[i]);
}

template <bool BYSEG>
__device__ inline int digit_of(const uint64_t *key, const int32_t *seg, int64_t i, int shift) {
  if (BYSEG) return (int)(((uint32_t)seg[i] >> shift) & (RDIG - 1));
  return (int)((key[i] >> shift) & (RDIG - 1));
}

// per-tile digit counts, digit-major: counts[d * ntiles + tile]
template <bool BYSEG>
__global__ void k_radix_count(const uint64_t *key, const int32_t *seg, int64_t n, int shift, int64_t ntiles,
                              int64_t *counts) {
  __shared__ int cnt[RDIG];
  if (threadIdx.x < RDIG) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RTILE + threadIdx.x * RITEMS;
  for (int j = 0; j < RITEMS; ++j)
    if (base + j < n) atomicAdd(&cnt[digit_of<BYSEG>(key, seg, base + j, shift)], 1);
  __syncthreads();
  if (threadIdx.x < RDIG) counts[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// stable scatter: thread t owns items [base, base + RITEMS) in order
template <bool BYSEG>
__global__ void k_radix_scatter(const uint64_t *key, const int32_t *seg, const int32_t *idx, int64_t n, int shift,
                                int64_t ntiles, const int64_t *offs, uint64_t *key2, int32_t *seg2, int32_t *idx2) {
  __shared__ int pre[RDIG][TPB];
  int local[RDIG];
#pragma unroll
  for (int d = 0; d < RDIG; ++d) local[d] = 0;
  const int64_t base = (int64_t)blockIdx.x * RTILE + threadIdx.x * RITEMS;
  for (int j = 0; j < RITEMS; ++j)
    if (base + j < n) local[digit_of<BYSEG>(key, seg, base + j, shift)]++;
#pragma unroll
  for (int d = 0; d < RDIG; ++d) pre[d][threadIdx.x] = local[d];
  __syncthreads();
  if (threadIdx.x < RDIG) {
    int run = 0;
    for (int t = 0; t < TPB; ++t) {
      const int v = pre[threadIdx.x][t];
      pre[threadIdx.x][t] = run;
      run += v;
    }
  }
  __syncthreads();
  int cur[RDIG];
#pragma unroll
  for (int d = 0; d < RDIG; ++d) cur[d] = 0;
  for (int j = 0; j < RITEMS; ++j) {
    const int64_t i = base + j;
    if (i >= n) break;
    const int d = digit_of<BYSEG>(key, seg, i, shift);
    int r = 0;
#pragma unroll
    for (int dd = 0; dd < RDIG; ++dd)
      if (dd == d) r = cur[dd]++;
    const int64_t o = offs[d * ntiles + blockIdx.x] + pre[d][threadIdx.x] + r;
    key2[o] = key[i];
    seg2[o] = seg[i];
    idx2[o] = idx[i];
  }
}

__global__ void k_seg_bounds(const int32_t *seg, int64_t n, int64_t *start, int64_t *end) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int s = seg[p];
  if (p == 0 || seg[p - 1] != s) start[s] = p;
  if (p == n - 1 || seg[p + 1] != s) end[s] = p + 1;
}

// sequential prefix per segment, in sorted order
__global__ void k_seg_select(const int32_t *idx, const int64_t *start, const int64_t *end, int nseg,
                             const double *nrm2, const double *budget, const double *segw, int64_t *keep,
                             double *seg_err, int64_t *seg_cnt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  double acc = 0.0;
  int64_t cnt = 0;
  const double bud = budget[s], wt = segw[s];
  for (int64_t p = start[s]; p < end[s]; ++p) {
    const int32_t b = idx[p];
    const double nxt = acc + wt * nrm2[b];
    if (nxt <= bud) {
      acc = nxt;
      keep[b] = 0;
      ++cnt;
    } else {
      break;
    }
  }
  seg_err[s] = acc;
  seg_cnt[s] = cnt;
}

// The same selection with one workgroup per segment, for few long segments
// (the Frobenius norm has one segment over the whole matrix): the squared
// norms of the next SEL candidates are gathered into LDS by all threads at
// once, and thread 0 adds them in sorted order exactly as k_seg_select does
// (same expression, same order, same stopping test), so the removed set and
// the segment error are the same bits; the gather latency is paid once per
// SEL candidates instead of once per candidate.
constexpr int SEL = 256;
__global__ __launch_bounds__(SEL) void k_seg_select_wg(const int32_t *idx, const int64_t *start, const int64_t *end,
                                                       int nseg, const double *nrm2, const double *budget,
                                                       const double *segw, int64_t *keep, double *seg_err,
                                                       int64_t *seg_cnt) {
  __shared__ double v[SEL];
  __shared__ int taken, stopped;
  const int s = blockIdx.x;
  if (s >= nseg) return;
  const int64_t p1 = end[s];
  const double bud = budget[s], wt = segw[s];
  double acc = 0.0;  // thread 0's running sum
  int64_t cnt = 0;
  for (int64_t base = start[s]; base < p1; base += SEL) {
    const int64_t p = base + threadIdx.x;
    if (p < p1) v[threadIdx.x] = nrm2[idx[p]];
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = (int)(p1 - base < SEL ? p1 - base : SEL);
      int t = 0;
      for (; t < n; ++t) {
        const double nxt = acc + wt * v[t];
        if (nxt <= bud)
          acc = nxt;
        else
          break;
      }
      cnt += t;
      taken = t;
      stopped = t < n ? 1 : 0;
    }
    __syncthreads();
    const int tk = taken;
    const bool stop = stopped != 0;
    if ((int)threadIdx.x < tk) keep[idx[p]] = 0;
    __syncthreads();  // taken / stopped and v are rewritten in the next round
    if (stop) break;
  }
  if (threadIdx.x == 0) {
    seg_err[s] = acc;
    seg_cnt[s] = cnt;
  }
}

__global__ void k_gather_rowptr(const int64_t *row_ptr, const int64_t *pos, int nbr, int64_t *out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I > nbr) return;
  out[I] = pos[row_ptr[I]];
}

__global__ void k_compact(const int64_t *keep, const int64_t *pos, int64_t nnzb, const int32_t *col,
                          const int32_t *row_of, const int32_t *slot, int32_t *col2, int32_t *row2, int32_t *slot2) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb || !keep[b]) return;
  const int64_t o = pos[b];
  col2[o] = col[b];
  row2[o] = row_of[b];
  slot2[o] = slot ? slot[b] : (int32_t)b;
}

__global__ void k_mark_in_mask(const int32_t *row_of, const int32_t *col, int64_t nnzb, const uint32_t *mbits, int W,
                               int64_t *keep) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int I = row_of[b], J = col[b];
  keep[b] = (mbits[(int64_t)I * W + (J >> 5)] >> (J & 31)) & 1u;
}

}  // namespace

void truncate_select(Ctx &c, const Pattern &pat, const double *nrm2, double tau, int norm, int64_t coarse_bs,
                     int64_t *keep, TruncOut &out, int nc_out[1]) {
  const int64_t nnzb = pat.nnzb;
  const int nbr = pat.nbr;
  out.seg_err.clear();
  out.removed = 0;
  nc_out[0] = 1;
  if (nnzb > 0) {
    k_fill_i64<<<blocks_for(nnzb), TPB, 0, c.stream>>>(keep, nnzb, 1);
    SP2_LAUNCH_CHECK();
  }
  if (norm == SP2_TRUNC_NONE || !(tau > 0.0) || nnzb == 0) return;

  // ---- segments and budgets ------------------------------------------------
  int cb, nc;
  std::vector<double> budget, segw;
  if (norm == SP2_TRUNC_FROB) {
    cb = nbr > 0 ? nbr : 1;
    nc = 1;
    budget.assign(1, tau * tau);
    segw.assign(1, 2.0);
  } else {
    if (coarse_bs <= 0 || coarse_bs % B != 0) fail(SP2_ERR_INVALID_ARG, "coarse_bs must be a positive multiple of 64");
    cb = (int)(coarse_bs / B);
    nc = (nbr + cb - 1) / cb;
    Buf occ = c.alloc(sizeof(int32_t) * (size_t)nc * nc);
    launch_fill_i32(c, occ.as<int32_t>(), (int64_t)nc * nc, 0);
    k_occupancy<<<blocks_for(nnzb), TPB, 0, c.stream>>>(pat.row_of.as<int32_t>(), pat.col_idx.as<int32_t>(), nnzb,
                                                          cb, nc, occ.as<int32_t>());
    SP2_LAUNCH_CHECK();
    std::vector<int32_t> h((size_t)nc * nc);
    c.d2h(h.data(), occ.p, h.size() * sizeof(int32_t));
    std::vector<int64_t> m(nc, 0);
    for (int R = 0; R < nc; ++R)
      for (int S = 0; S < nc; ++S) m[R] += h[(size_t)R * nc + S];
    budget.assign((size_t)nc * nc, 0.0);
    segw.assign((size_t)nc * nc, 1.0);
    for (int R = 0; R < nc; ++R)
      for (int S = R; S < nc; ++S) {
        const int64_t mm = m[R] > m[S] ? m[R] : m[S];
        const double beta = mm > 0 ? tau / (double)mm : 0.0;
        budget[(size_t)R * nc + S] = beta * beta;
        segw[(size_t)R * nc + S] = (R == S) ? 2.0 : 1.0;
      }
  }
  nc_out[0] = nc;
  const int nseg = nc * nc;
  Buf d_budget = c.alloc(sizeof(double) * nseg), d_segw = c.alloc(sizeof(double) * nseg);
  c.h2d(d_budget.p, budget.data(), sizeof(double) * nseg);
  c.h2d(d_segw.p, segw.data(), sizeof(double) * nseg);

  // ---- candidates ----------------------------------------------------------
  Buf flag = c.alloc(sizeof(int64_t) * nnzb), pos = c.alloc(sizeof(int64_t) * (nnzb + 1));
  k_cand_flag<<<blocks_for(nnzb), TPB, 0, c.stream>>>(pat.row_of.as<int32_t>(), pat.col_idx.as<int32_t>(), nnzb,
                                                        nrm2, cb, nc, d_budget.as<double>(), d_segw.as<double>(),
                                                        flag.as<int64_t>());
  SP2_LAUNCH_CHECK();
  scan_exclusive_i64(c, flag.as<int64_t>(), pos.as<int64_t>(), nnzb);
  int64_t ncand = 0;
  c.d2h(&ncand, pos.as<int64_t>() + nnzb, sizeof(int64_t));
  out.seg_err.assign(nseg, 0.0);
  if (ncand == 0) return;

  Buf k0 = c.alloc(8 * ncand), k1 = c.alloc(8 * ncand);
  Buf s0 = c.alloc(4 * ncand), s1 = c.alloc(4 * ncand);
  Buf i0 = c.alloc(4 * ncand), i1 = c.alloc(4 * ncand);
  k_cand_write<<<blocks_for(nnzb), TPB, 0, c.stream>>>(pat.row_of.as<int32_t>(), pat.col_idx.as<int32_t>(), nnzb,
                                                         nrm2, cb, nc, flag.as<int64_t>(), pos.as<int64_t>(),
                                                         k0.as<uint64_t>(), s0.as<int32_t>(), i0.as<int32_t>());
  SP2_LAUNCH_CHECK();

  // ---- stable LSD radix sort by (segment, norm^2) ------------------------------
  Buf rng = c.alloc(32);
  {
    struct R {
      unsigned long long kor, kand;
      unsigned int sor, sand;
    } r0{0ull, ~0ull, 0u, ~0u};
    c.h2d(rng.p, &r0, sizeof(r0));
    unsigned char *base = rng.as<unsigned char>();
    k_bits_range<<<blocks_for(ncand), TPB, 0, c.stream>>>(
        k0.as<uint64_t>(), s0.as<int32_t>(), ncand, (unsigned long long *)base, (unsigned long long *)(base + 8),
        (unsigned int *)(base + 16), (unsigned int *)(base + 20));
    SP2_LAUNCH_CHECK();
    c.d2h(&r0, rng.p, sizeof(r0));
    const uint64_t kvar = r0.kor ^ r0.kand;
    const uint32_t svar = r0.sor ^ r0.sand;
    const int64_t ntiles = (ncand + RTILE - 1) / RTILE;
    Buf counts = c.alloc(sizeof(int64_t) * RDIG * ntiles), offs = c.alloc(sizeof(int64_t) * (RDIG * ntiles + 1));
    uint64_t *ka = k0.as<uint64_t>(), *kb = k1.as<uint64_t>();
    int32_t *sa = s0.as<int32_t>(), *sb = s1.as<int32_t>(), *ia = i0.as<int32_t>(), *ib = i1.as<int32_t>();
    auto pass = [&](bool byseg, int shift) {
      if (byseg) {
        k_radix_count<true><<<(unsigned)ntiles, TPB, 0, c.stream>>>(ka, sa, ncand, shift, ntiles,
                                                                    counts.as<int64_t>());
      } else {
        k_radix_count<false><<<(unsigned)ntiles, TPB, 0, c.stream>>>(ka, sa, ncand, shift, ntiles,
                                                                     counts.as<int64_t>());
      }
      SP2_LAUNCH_CHECK();
      scan_exclusive_i64(c, counts.as<int64_t>(), offs.as<int64_t>(), RDIG * ntiles);
      if (byseg) {
        k_radix_scatter<true><<<(unsigned)ntiles, TPB, 0, c.stream>>>(ka, sa, ia, ncand, shift, ntiles,
                                                                      offs.as<int64_t>(), kb, sb, ib);
      } else {
        k_radix_scatter<false><<<(unsigned)ntiles, TPB, 0, c.stream>>>(ka, sa, ia, ncand, shift, ntiles,
                                                                       offs.as<int64_t>(), kb, sb, ib);
      }
      SP2_LAUNCH_CHECK();
      std::swap(ka, kb);
      std::swap(sa, sb);
      std::swap(ia, ib);
    };
    for (int sh = 0; sh < 64; sh += RBITS)
      if ((kvar >> sh) & (RDIG - 1)) pass(false, sh);
    for (int sh = 0; sh < 32; sh += RBITS)
      if ((svar >> sh) & (RDIG - 1)) pass(true, sh);

    // ---- per-segment prefixes ---------------------------------------------------
    Buf st = c.alloc(sizeof(int64_t) * nseg), en = c.alloc(sizeof(int64_t) * nseg);
    k_fill_i64<<<blocks_for(nseg), TPB, 0, c.stream>>>(st.as<int64_t>(), nseg, 0);
    k_fill_i64<<<blocks_for(nseg), TPB, 0, c.stream>>>(en.as<int64_t>(), nseg, 0);
    SP2_LAUNCH_CHECK();
    k_seg_bounds<<<blocks_for(ncand), TPB, 0, c.stream>>>(sa, ncand, st.as<int64_t>(), en.as<int64_t>());
    SP2_LAUNCH_CHECK();
    Buf serr = c.alloc(sizeof(double) * nseg), scnt = c.alloc(sizeof(int64_t) * nseg);
    // few segments (the Frobenius norm, coarse Frob-Inf partitions): a
    // workgroup each; many short ones: a thread each (same result)
    if (nseg <= 16384)
      k_seg_select_wg<<<(unsigned)nseg, SEL, 0, c.stream>>>(ia, st.as<int64_t>(), en.as<int64_t>(), nseg, nrm2,
                                                             d_budget.as<double>(), d_segw.as<double>(), keep,
                                                             serr.as<double>(), scnt.as<int64_t>());
    else
      k_seg_select<<<blocks_for(nseg, 64), 64, 0, c.stream>>>(ia, st.as<int64_t>(), en.as<int64_t>(), nseg, nrm2,
                                                               d_budget.as<double>(), d_segw.as<double>(), keep,
                                                               serr.as<double>(), scnt.as<int64_t>());
    SP2_LAUNCH_CHECK();
    std::vector<int64_t> cnt(nseg);
    c.d2h(out.seg_err.data(), serr.p, sizeof(double) * nseg);
    c.d2h(cnt.data(), scnt.p, sizeof(int64_t) * nseg);
    for (int s = 0; s < nseg; ++s) out.removed += cnt[s];
  }
}

void compact_pattern(Ctx &c, const Pattern &in, const int64_t *keep, Pattern &out) {
  const int64_t nnzb = in.nnzb;
  Buf pos = c.alloc(sizeof(int64_t) * (nnzb + 1));
  scan_exclusive_i64(c, keep, pos.as<int64_t>(), nnzb);
  int64_t nn = 0;
  c.d2h(&nn, pos.as<int64_t>() + nnzb, sizeof(int64_t));
  out.n = in.n;
  out.nbr = in.nbr;
  out.nnzb = nn;
  out.row_ptr = c.alloc(sizeof(int64_t) * (in.nbr + 1));
  out.col_idx = c.alloc(sizeof(int32_t) * (nn > 0 ? nn : 1));
  out.row_of = c.alloc(sizeof(int32_t) * (nn > 0 ? nn : 1));
  out.slot = c.alloc(sizeof(int32_t) * (nn > 0 ? nn : 1));
  k_gather_rowptr<<<blocks_for(in.nbr + 1), TPB, 0, c.stream>>>(in.row_ptr.as<int64_t>(), pos.as<int64_t>(), in.nbr,
                                                                 out.row_ptr.as<int64_t>());
  SP2_LAUNCH_CHECK();
  if (nnzb > 0) {
    k_compact<<<blocks_for(nnzb), TPB, 0, c.stream>>>(keep, pos.as<int64_t>(), nnzb, in.col_idx.as<int32_t>(),
                                                        in.row_of.as<int32_t>(), in.slot.as<int32_t>(),
                                                        out.col_idx.as<int32_t>(), out.row_of.as<int32_t>(),
                                                        out.slot.as<int32_t>());
    SP2_LAUNCH_CHECK();
  }
}

void launch_mark_in_mask(Ctx &c, const Pattern &pat, const uint32_t *mask_bits, int W, int64_t *keep) {
  if (pat.nnzb <= 0) return;
  k_mark_in_mask<<<blocks_for(pat.nnzb), TPB, 0, c.stream>>>(pat.row_of.as<int32_t>(), pat.col_idx.as<int32_t>(),
                                                               pat.nnzb, mask_bits, W, keep);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
