// Value kernels: finiteness check, Gershgorin bounds (Step 1), block gathers
// and precision conversion, deterministic reductions of per-block partial
// sums (traces and Frobenius norms of Algorithms 1 and 2), block norms for
// truncation, and the separate polynomial update used by the trace-correcting
// run (where p_i is only known after the traces of the square).
#include "internal.h"

namespace sp2 {

namespace {

constexpr int TPB = 256;
constexpr int RED_BLOCKS = 256;  // fixed, so reductions are reproducible on any device
static_assert(reduce_stage_doubles(1) == RED_BLOCKS, "staging size of launch_reduce_parts");

__global__ void k_check_finite(const double *v, int64_t n, int32_t *flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) atomicOr(flag, 1);
}

// Row sums of |F_ij| over the full symmetric matrix for the 64 rows of block
// row I.  Four groups of 64 threads take every fourth neighbour block; the
// group sums are added in a fixed order.
__global__ void k_gershgorin(const int32_t *idxmap, const int64_t *adj_ptr, const int32_t *adj_col,
                             const double *val, int nbr, int64_t n, double *row_lo, double *row_hi) {
  __shared__ double part[4][64];
  __shared__ double dg[64];
  __shared__ double lo_s[64], hi_s[64];
  const int I = blockIdx.x;
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  if (threadIdx.x < 64) dg[r] = 0.0;
  __syncthreads();
  double s = 0.0;
  for (int64_t k = adj_ptr[I] + g; k < adj_ptr[I + 1]; k += 4) {
    const int K = adj_col[k];
    const int32_t sl = idxmap[(int64_t)I * nbr + K];
    if (sl < 0) continue;
    const double *blk = val + (int64_t)sl * BB;
    if (K >= I) {
      for (int c = 0; c < 64; ++c) s += fabs(blk[r * 64 + c]);
      if (K == I) dg[r] = blk[r * 64 + r];
    } else {
      for (int c = 0; c < 64; ++c) s += fabs(blk[c * 64 + r]);
    }
  }
  part[g][r] = s;
  __syncthreads();
  if (threadIdx.x < 64) {
    const double t = ((part[0][r] + part[1][r]) + part[2][r]) + part[3][r];
    const double d = dg[r];
    const double rad = t - fabs(d);
    const bool real = (int64_t)I * 64 + r < n;
    lo_s[r] = real ? d - rad : INFINITY;
    hi_s[r] = real ? d + rad : -INFINITY;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < 64; ++i) {
      lo = fmin(lo, lo_s[i]);
      hi = fmax(hi, hi_s[i]);
    }
    row_lo[I] = lo;
    row_hi[I] = hi;
  }
}

__global__ void k_minmax(const double *lo, const double *hi, int n, double *out2) {
  __shared__ double a[TPB], b[TPB];
  double l = INFINITY, h = -INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    l = fmin(l, lo[i]);
    h = fmax(h, hi[i]);
  }
  a[threadIdx.x] = l;
  b[threadIdx.x] = h;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + o]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = a[0];
    out2[1] = b[0];
  }
}

template <typename S, typename D>
__global__ void k_gather(const S *src, const int32_t *slot, int64_t nblocks, D *dst) {
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t s = slot ? slot[b] : b;
  const S *in = src + s * BB;
  D *out = dst + b * BB;
  for (int e = threadIdx.x; e < BB; e += blockDim.x) out[e] = (D)in[e];
}

// out block b = a A_(I,J) + b B_(I,J) for the output block (I, J) = (row_of[b], col[b]);
// an operand without the block contributes zero
template <typename SA, typename SB>
__global__ void k_add_union(const int32_t *row_of, const int32_t *col, int64_t nblocks, int nbr, const SA *pa,
                            const int32_t *ia, double a, const SB *pb, const int32_t *ib, double b, double *out) {
  const int64_t o = blockIdx.x;
  if (o >= nblocks) return;
  const int64_t k = (int64_t)row_of[o] * nbr + col[o];
  const int32_t sa = ia[k], sb = ib[k];
  double *ob = out + o * BB;
  for (int e = threadIdx.x; e < BB; e += blockDim.x) {
    double v = 0.0;
    if (sa >= 0) v += a * (double)pa[(int64_t)sa * BB + e];
    if (sb >= 0) v += b * (double)pb[(int64_t)sb * BB + e];
    ob[e] = v;
  }
}

// block norms^2 weighted for the whole symmetric matrix: x2 off the diagonal
__global__ void k_weight_offdiag(double *nrm2, const int32_t *row_of, const int32_t *col, int64_t nblocks) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b < nblocks && row_of[b] != col[b]) nrm2[b] *= 2.0;
}

// diagonal blocks made exactly symmetric, (B + B^T) / 2 (sign = 1), or
// antisymmetric, (B - B^T) / 2 (sign = -1): a square computes the (r, c) and
// (c, r) entries of a diagonal block separately, so they differ by rounding.
// The diagonal block (I, I), when stored, is the first block of row I.
template <typename T>
__global__ void k_sym_diag(T *pool, const int64_t *row_ptr, const int32_t *col_idx, const int32_t *slot, int nbr,
                           double sign) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  const int64_t b = row_ptr[I];
  if (b >= row_ptr[I + 1] || col_idx[b] != I) return;
  T *blk = pool + (int64_t)(slot ? slot[b] : b) * BB;
  for (int e = threadIdx.x; e < BB; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    if (r < c) {
      const double m = 0.5 * ((double)blk[r * 64 + c] + sign * (double)blk[c * 64 + r]);
      blk[r * 64 + c] = (T)m;
      blk[c * 64 + r] = (T)(sign * m);
    } else if (r == c && sign < 0.0) {
      blk[e] = (T)0;
    }
  }
}

// deterministic sum over rows of a [nrows][ncols] array (ncols <= 8)
__device__ double block_sum(double v) {
  __shared__ double sh[TPB / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < TPB / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ void k_reduce_stage1(const double *parts, int64_t nrows, int ncols, double *stage) {
  const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * chunk, r1 = min(nrows, r0 + chunk);
  for (int j = 0; j < ncols; ++j) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += parts[r * ncols + j];
    const double t = block_sum(s);
    if (threadIdx.x == 0) stage[blockIdx.x * ncols + j] = t;
  }
}

__global__ void k_reduce_stage2(const double *stage, int nstage, int ncols, double *out) {
  for (int j = 0; j < ncols; ++j) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nstage; i += blockDim.x) s += stage[i * ncols + j];
    const double t = block_sum(s);
    if (threadIdx.x == 0) out[j] = t;
  }
}

template <typename T>
__global__ void k_block_norms(const T *pool, const int32_t *slot, int64_t nblocks, double *nrm2) {
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t s = slot ? slot[b] : b;
  double acc = 0.0;
  for (int e = threadIdx.x; e < BB; e += blockDim.x) {
    const double v = (double)pool[s * BB + e];
    acc += v * v;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) nrm2[b] = t;
}

// out = ca I + cb X + cc S on the pattern of S (in place in the S pool);
// parts[w * NPART + 3] receives ||out_w||_F^2.
template <typename TX, typename TS>
__global__ void k_update(const TX *xpool, const int32_t *xidxmap, int nbr, const int32_t *out_row,
                         const int32_t *out_col, int64_t nout, TS *spool, double ca, double cb, double cc, int64_t n,
                         double *parts) {
  const int64_t w = blockIdx.x;
  if (w >= nout) return;
  const int I = out_row[w], J = out_col[w];
  const int32_t sx = xidxmap[(int64_t)I * nbr + J];
  double acc = 0.0;
  for (int e = threadIdx.x; e < BB; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    const double x = sx >= 0 ? (double)xpool[(int64_t)sx * BB + e] : 0.0;
    const double s = (double)spool[w * BB + e];
    const bool d = (I == J) && (r == c) && ((int64_t)I * B + r < n);
    const double o = cc * s + cb * x + (d ? ca : 0.0);
    spool[w * BB + e] = (TS)o;
    const double ov = (double)(TS)o;
    acc += ov * ov;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) parts[w * NPART + 3] = t;
}

// Frob-Inf mixed norm (section "Upper bounds for the spectral norm") of a
// symmetric matrix held by its upper blocks, in two deterministic passes.
// Coarse submatrices are cb x cb blocks; coarse (R, S), R <= S, gets the
// squared Frobenius norm of its part of the full matrix: inside a diagonal
// coarse submatrix an off-diagonal block stands for itself and its mirror
// (weight 2), elsewhere each stored block counts once (its mirror lies in
// (S, R)).  One thread per upper coarse pair sums, row by row, the blocks
// whose column falls in S's range (a contiguous run of the sorted row).
__global__ void k_coarse_pairs(const int64_t *row_ptr, const int32_t *col_idx, const double *nrm2, int nbr, int cb,
                               int nc, int64_t npairs, double *pair) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= npairs) return;
  // q -> (R, S) with R <= S, row-major over the upper triangle of nc x nc:
  // row R starts at P(R) = R (2 nc - R + 1) / 2
  auto start = [nc](int64_t r) { return r * (2 * (int64_t)nc - r + 1) / 2; };
  const double d = 2.0 * nc + 1.0;
  int64_t R = (int64_t)((d - sqrt(fmax(d * d - 8.0 * (double)q, 0.0))) / 2.0);
  R = R < 0 ? 0 : (R >= nc ? nc - 1 : R);
  while (R > 0 && start(R) > q) --R;
  while (R + 1 < nc && start(R + 1) <= q) ++R;
  const int S = (int)(R + (q - start(R)));
  const int jlo = S * cb, jhi = min(nbr, (S + 1) * cb);
  double sum = 0.0;
  for (int I = (int)R * cb; I < min(nbr, ((int)R + 1) * cb); ++I) {
    int64_t lo = row_ptr[I], hi = row_ptr[I + 1];
    // first position with col >= jlo
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (col_idx[mid] < jlo) lo = mid + 1;
      else hi = mid;
    }
    for (int64_t b = lo; b < row_ptr[I + 1] && col_idx[b] < jhi; ++b)
      sum += (R == S && col_idx[b] != I) ? 2.0 * nrm2[b] : nrm2[b];
  }
  pair[q] = sum;
}

// row sums of the coarse Frobenius norms: rowsum[R] = sum_S sqrt(c(R, S)),
// c symmetric, read from the packed upper triangle
__global__ void k_coarse_rowsum(const double *pair, int nc, double *rowsum) {
  const int R = blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nc) return;
  double s = 0.0;
  for (int S = 0; S < nc; ++S) {
    const int a = min(R, S), b = max(R, S);
    const int64_t q = (int64_t)a * nc - (int64_t)a * (a - 1) / 2 + (b - a);
    s += sqrt(pair[q]);
  }
  rowsum[R] = s;
}

}  // namespace

void launch_check_finite(Ctx &c, const double *v, int64_t n, int32_t *flag) {
  if (n <= 0) return;
  int64_t g = (n + TPB - 1) / TPB;
  if (g > 4096) g = 4096;
  k_check_finite<<<(unsigned)g, TPB, 0, c.stream>>>(v, n, flag);
  SP2_LAUNCH_CHECK();
}

void launch_gershgorin(Ctx &c, const int32_t *idxmap, const int64_t *adj_ptr, const int32_t *adj_col,
                       const double *val, int nbr, int64_t n, double *row_lo, double *row_hi) {
  if (nbr <= 0) return;
  k_gershgorin<<<nbr, TPB, 0, c.stream>>>(idxmap, adj_ptr, adj_col, val, nbr, n, row_lo, row_hi);
  SP2_LAUNCH_CHECK();
}

void launch_minmax(Ctx &c, const double *lo, const double *hi, int n, double *out2) {
  k_minmax<<<1, TPB, 0, c.stream>>>(lo, hi, n, out2);
  SP2_LAUNCH_CHECK();
}

void launch_gather(Ctx &c, const void *src, int src_prec, const int32_t *slot, int64_t nblocks, void *dst,
                   int dst_prec) {
  if (nblocks <= 0) return;
  const unsigned g = (unsigned)nblocks;
  if (src_prec == P64 && dst_prec == P64)
    k_gather<double, double><<<g, TPB, 0, c.stream>>>((const double *)src, slot, nblocks, (double *)dst);
  else if (src_prec == P64 && dst_prec == P32)
    k_gather<double, float><<<g, TPB, 0, c.stream>>>((const double *)src, slot, nblocks, (float *)dst);
  else if (src_prec == P32 && dst_prec == P64)
    k_gather<float, double><<<g, TPB, 0, c.stream>>>((const float *)src, slot, nblocks, (double *)dst);
  else
    k_gather<float, float><<<g, TPB, 0, c.stream>>>((const float *)src, slot, nblocks, (float *)dst);
  SP2_LAUNCH_CHECK();
}

void launch_add_union(Ctx &c, const int32_t *row_of, const int32_t *col, int64_t nblocks, int nbr, const void *pa,
                      int preca, const int32_t *ia, double a, const void *pb, int precb, const int32_t *ib, double b,
                      double *out) {
  if (nblocks <= 0) return;
  const unsigned g = (unsigned)nblocks;
  if (preca == P64 && precb == P64)
    k_add_union<double, double><<<g, TPB, 0, c.stream>>>(row_of, col, nblocks, nbr, (const double *)pa, ia, a,
                                                         (const double *)pb, ib, b, out);
  else if (preca == P64 && precb == P32)
    k_add_union<double, float><<<g, TPB, 0, c.stream>>>(row_of, col, nblocks, nbr, (const double *)pa, ia, a,
                                                        (const float *)pb, ib, b, out);
  else if (preca == P32 && precb == P64)
    k_add_union<float, double><<<g, TPB, 0, c.stream>>>(row_of, col, nblocks, nbr, (const float *)pa, ia, a,
                                                        (const double *)pb, ib, b, out);
  else
    k_add_union<float, float><<<g, TPB, 0, c.stream>>>(row_of, col, nblocks, nbr, (const float *)pa, ia, a,
                                                       (const float *)pb, ib, b, out);
  SP2_LAUNCH_CHECK();
}

void launch_weight_offdiag(Ctx &c, double *nrm2, const int32_t *row_of, const int32_t *col, int64_t nblocks) {
  if (nblocks <= 0) return;
  k_weight_offdiag<<<(unsigned)((nblocks + TPB - 1) / TPB), TPB, 0, c.stream>>>(nrm2, row_of, col, nblocks);
  SP2_LAUNCH_CHECK();
}

void launch_sym_diag(Ctx &c, void *pool, int prec, const int64_t *row_ptr, const int32_t *col_idx,
                     const int32_t *slot, int nbr, double sign) {
  if (nbr <= 0) return;
  if (prec == P64)
    k_sym_diag<double><<<(unsigned)nbr, TPB, 0, c.stream>>>((double *)pool, row_ptr, col_idx, slot, nbr, sign);
  else
    k_sym_diag<float><<<(unsigned)nbr, TPB, 0, c.stream>>>((float *)pool, row_ptr, col_idx, slot, nbr, sign);
  SP2_LAUNCH_CHECK();
}

void launch_reduce_parts(Ctx &c, const double *parts, int64_t nrows, int ncols, double *out, double *stage) {
  k_reduce_stage1<<<RED_BLOCKS, TPB, 0, c.stream>>>(parts, nrows, ncols, stage);
  SP2_LAUNCH_CHECK();
  k_reduce_stage2<<<1, TPB, 0, c.stream>>>(stage, RED_BLOCKS, ncols, out);
  SP2_LAUNCH_CHECK();
}

void launch_reduce_parts(Ctx &c, const double *parts, int64_t nrows, int ncols, double *out) {
  Buf stage = c.alloc(sizeof(double) * RED_BLOCKS * ncols);
  launch_reduce_parts(c, parts, nrows, ncols, out, stage.as<double>());
}

void launch_block_norms(Ctx &c, const void *pool, int prec, const int32_t *slot, int64_t nblocks, double *nrm2) {
  if (nblocks <= 0) return;
  if (prec == P64)
    k_block_norms<double><<<(unsigned)nblocks, TPB, 0, c.stream>>>((const double *)pool, slot, nblocks, nrm2);
  else
    k_block_norms<float><<<(unsigned)nblocks, TPB, 0, c.stream>>>((const float *)pool, slot, nblocks, nrm2);
  SP2_LAUNCH_CHECK();
}

void launch_update(Ctx &c, const void *xpool, int xprec, const int32_t *xidxmap, int nbr, const int32_t *out_row,
                   const int32_t *out_col, int64_t nout, void *spool, int sprec, double ca, double cb, double cc,
                   int64_t n, double *parts) {
  if (nout <= 0) return;
  const unsigned g = (unsigned)nout;
  if (xprec == P64 && sprec == P64)
    k_update<double, double><<<g, TPB, 0, c.stream>>>((const double *)xpool, xidxmap, nbr, out_row, out_col, nout,
                                                      (double *)spool, ca, cb, cc, n, parts);
  else if (xprec == P32 && sprec == P32)
    k_update<float, float><<<g, TPB, 0, c.stream>>>((const float *)xpool, xidxmap, nbr, out_row, out_col, nout,
                                                    (float *)spool, ca, cb, cc, n, parts);
  else
    fail(SP2_ERR_INVALID_ARG, "update: mixed pool precisions");
  SP2_LAUNCH_CHECK();
}

void launch_coarse_rowsums(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, const double *nrm2, int nbr,
                           int cb, int nc, double *pair, double *rowsum) {
  if (nc <= 0) return;
  const int64_t npairs = (int64_t)nc * (nc + 1) / 2;
  k_coarse_pairs<<<(unsigned)((npairs + TPB - 1) / TPB), TPB, 0, c.stream>>>(row_ptr, col_idx, nrm2, nbr, cb, nc,
                                                                             npairs, pair);
  SP2_LAUNCH_CHECK();
  k_coarse_rowsum<<<(unsigned)((nc + TPB - 1) / TPB), TPB, 0, c.stream>>>(pair, nc, rowsum);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
