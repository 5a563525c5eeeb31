// Block-pattern kernels: validation, dense block maps, symbolic planning of
// the block pattern of X^2, prefix scans and the pattern of X_0.
//
// The symbolic step realises the block-level structure of the square in
// Algorithm 2: for a symmetric X stored as its upper triangle, S = X^2 has a
// block (I, J) exactly when some K has X_IK and X_KJ stored; only I <= J is
// produced (section "Implementation details": symmetric matrices keep the
// upper triangle).  Block triples are never materialised: the numeric kernel
// intersects the bit rows of I and J on the fly.
#include "internal.h"

namespace sp2 {

namespace {

constexpr int TPB = 256;

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// one block per block row
__global__ void k_row_of(const int64_t *row_ptr, int nbr, int32_t *row_of) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  for (int64_t b = row_ptr[I] + threadIdx.x; b < row_ptr[I + 1]; b += blockDim.x) row_of[b] = I;
}

// flag bit 1: column out of range / below diagonal; bit 2: not strictly increasing;
// bit 4: row_ptr not monotone
__global__ void k_validate(const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb, int32_t *flag) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  const int64_t s = row_ptr[I], e = row_ptr[I + 1];
  if (threadIdx.x == 0 && (s > e || s < 0 || e > nnzb)) atomicOr(flag, 4);
  if (s > e || s < 0 || e > nnzb) return;
  for (int64_t b = s + threadIdx.x; b < e; b += blockDim.x) {
    const int32_t c = col_idx[b];
    if (c < I || c >= nbr) atomicOr(flag, 1);
    if (b > s && col_idx[b - 1] >= c) atomicOr(flag, 2);
  }
}

__global__ void k_build_maps(const int32_t *row_of, const int32_t *col_idx, const int32_t *slot, int64_t nnzb,
                             int nbr, int W, int32_t *idxmap, uint32_t *bits) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int I = row_of[b], K = col_idx[b];
  const int32_t s = slot ? slot[b] : (int32_t)b;
  idxmap[(int64_t)I * nbr + K] = s;
  idxmap[(int64_t)K * nbr + I] = s;
  atomicOr(&bits[(int64_t)I * W + (K >> 5)], 1u << (K & 31));
  if (K != I) atomicOr(&bits[(int64_t)K * W + (I >> 5)], 1u << (I & 31));
}

// deterministic block-wide exclusive scan of one int64 per thread (blockDim = TPB)
__device__ int64_t block_exscan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[TPB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up((long long)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int64_t base = 0, tot = 0;
  for (int i = 0; i < TPB / 64; ++i) {
    if (i < wv) base += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ void k_popcount_rows(const uint32_t *bits, int nbr, int W, int64_t *counts) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  int64_t c = 0;
  for (int w = threadIdx.x; w < W; w += blockDim.x) c += __popc(bits[(int64_t)I * W + w]);
  int64_t tot;
  block_exscan(c, &tot);
  if (threadIdx.x == 0) counts[I] = tot;
}

// set bits of row I, in increasing order, to cols[ptr[I] ..]; rows (optional) gets I
__global__ void k_extract_rows(const uint32_t *bits, int nbr, int W, const int64_t *ptr, int32_t *cols,
                               int32_t *rows) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  const int wpt = (W + TPB - 1) / TPB;
  const int w0 = threadIdx.x * wpt, w1 = min(W, w0 + wpt);
  int64_t c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bits[(int64_t)I * W + w]);
  int64_t tot;
  int64_t off = block_exscan(c, &tot) + ptr[I];
  for (int w = w0; w < w1; ++w) {
    uint32_t m = bits[(int64_t)I * W + w];
    while (m) {
      const int bt = __builtin_ctz(m);
      m &= m - 1;
      cols[off] = w * 32 + bt;
      if (rows) rows[off] = I;
      ++off;
    }
  }
}

// outbits[I] = OR over K in adj(I) of bits[K], restricted to columns J >= I
// when upper (symmetric storage), every column otherwise (general storage).
__global__ void k_symbolic(const uint32_t *bits, const int64_t *adj_ptr, const int32_t *adj_col, int nbr, int W,
                           int WP, uint32_t *outbits, const uint32_t *bits2, const int64_t *adj_ptr2,
                           const int32_t *adj_col2, bool upper) {
  __shared__ uint32_t sh[TPB];
  const int I = blockIdx.x;
  if (I >= nbr) return;
  const int G = TPB / WP;
  const int wl = threadIdx.x % WP, g = threadIdx.x / WP;
  const int64_t k0 = adj_ptr[I], k1 = adj_ptr[I + 1];
  for (int wb = 0; wb < W; wb += WP) {
    const int w = wb + wl;
    uint32_t acc = 0;
    if (w < W) {
      for (int64_t k = k0 + g; k < k1; k += G) acc |= bits[(int64_t)adj_col[k] * W + w];
      if (bits2)
        for (int64_t k = adj_ptr2[I] + g; k < adj_ptr2[I + 1]; k += G) acc |= bits2[(int64_t)adj_col2[k] * W + w];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (g == 0 && w < W) {
      for (int gg = 1; gg < G; ++gg) acc |= sh[gg * WP + wl];
      const int lo = w * 32;
      if (upper) {
        if (lo + 32 <= I)
          acc = 0;
        else if (lo < I)
          acc &= ~((1u << (I - lo)) - 1u);
      }
      outbits[(int64_t)I * W + w] = acc;
    }
    __syncthreads();
  }
}

// upper part (J >= I) of the union of two symmetric block-row bitmaps
__global__ void k_or_upper(const uint32_t *a, const uint32_t *b, int nbr, int W, uint32_t *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)nbr * W) return;
  const int I = (int)(i / W), w = (int)(i % W);
  uint32_t v = a[i] | b[i];
  const int lo = w * 32;
  if (lo + 32 <= I)
    v = 0u;
  else if (lo < I)
    v &= ~((1u << (I - lo)) - 1u);
  out[i] = v;
}

// ---- 3-phase exclusive scan --------------------------------------------------
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;

__global__ void k_scan_tiles(const int64_t *in, int64_t n, int64_t *tsum) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  int64_t tot;
  block_exscan(s, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// single block: exclusive scan of ntiles tile sums, in place; writes total to *total
__global__ void k_scan_top(int64_t *tsum, int64_t ntiles, int64_t *total) {
  int64_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += TPB) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < ntiles ? tsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_exscan(v, &tot);
    if (i < ntiles) tsum[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_apply(const int64_t *in, int64_t n, const int64_t *toff, int64_t *out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t off = block_exscan(s, &tot) + toff[blockIdx.x];
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = off;
    off += v[i];
  }
}

// ---- X_0 pattern: F's pattern plus any missing diagonal block -------------
__global__ void k_diag_missing(const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t *counts) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr) return;
  const int64_t s = row_ptr[I], e = row_ptr[I + 1];
  const bool has = (e > s) && col_idx[s] == I;
  counts[I] = (e - s) + (has ? 0 : 1);
}

__global__ void k_x0_pattern(const int64_t *frow_ptr, const int32_t *fcol, int nbr, const int64_t *xrow_ptr,
                             int32_t *xcol, int32_t *src) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr) return;
  const int64_t s = frow_ptr[I], e = frow_ptr[I + 1];
  int64_t o = xrow_ptr[I];
  const bool has = (e > s) && fcol[s] == I;
  if (!has) {
    xcol[o] = I;
    src[o] = -1;
    ++o;
  }
  for (int64_t b = s; b < e; ++b, ++o) {
    xcol[o] = fcol[b];
    src[o] = (int32_t)b;
  }
}

// X_0 = (lmax I - F) / w (Algorithm 1), one block of 256 threads per 64 x 64 block
__global__ void k_init_x0(const double *fval, const int32_t *src, const int32_t *xrow_of, const int32_t *xcol,
                          int64_t nnzb, int64_t n, double lmax, double w, double *xval) {
  const int64_t b = blockIdx.x;
  if (b >= nnzb) return;
  const int I = xrow_of[b], J = xcol[b];
  const int32_t s = src[b];
  for (int e = threadIdx.x; e < BB; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    const double f = s >= 0 ? fval[(int64_t)s * BB + e] : 0.0;
    const bool d = (I == J) && (r == c) && ((int64_t)I * B + r < n);
    xval[b * BB + e] = ((d ? lmax : 0.0) - f) / w;
  }
}

inline int grid_for(int64_t n, int tpb = TPB) {
  int64_t g = (n + tpb - 1) / tpb;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

void launch_fill_i32(Ctx &c, int32_t *p, int64_t n, int32_t v) {
  if (n <= 0) return;
  k_fill_i32<<<grid_for(n), TPB, 0, c.stream>>>(p, n, v);
  SP2_LAUNCH_CHECK();
}
void launch_fill_u32(Ctx &c, uint32_t *p, int64_t n, uint32_t v) {
  if (n <= 0) return;
  k_fill_u32<<<grid_for(n), TPB, 0, c.stream>>>(p, n, v);
  SP2_LAUNCH_CHECK();
}
void launch_fill_f64(Ctx &c, double *p, int64_t n, double v) {
  if (n <= 0) return;
  k_fill_f64<<<grid_for(n), TPB, 0, c.stream>>>(p, n, v);
  SP2_LAUNCH_CHECK();
}
void launch_iota_i32(Ctx &c, int32_t *p, int64_t n) {
  if (n <= 0) return;
  k_iota_i32<<<grid_for(n), TPB, 0, c.stream>>>(p, n);
  SP2_LAUNCH_CHECK();
}
void launch_row_of(Ctx &c, const int64_t *row_ptr, int nbr, int32_t *row_of) {
  if (nbr <= 0) return;
  k_row_of<<<nbr, TPB, 0, c.stream>>>(row_ptr, nbr, row_of);
  SP2_LAUNCH_CHECK();
}
void launch_validate_pattern(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb,
                             int32_t *flag) {
  if (nbr <= 0) return;
  k_validate<<<nbr, TPB, 0, c.stream>>>(row_ptr, col_idx, nbr, nnzb, flag);
  SP2_LAUNCH_CHECK();
}
void launch_build_maps(Ctx &c, const int32_t *row_of, const int32_t *col_idx, const int32_t *slot, int64_t nnzb,
                       int nbr, int W, int32_t *idxmap, uint32_t *bits) {
  launch_fill_i32(c, idxmap, (int64_t)nbr * nbr, -1);
  launch_fill_u32(c, bits, (int64_t)nbr * W, 0u);
  if (nnzb <= 0) return;
  k_build_maps<<<(unsigned)((nnzb + TPB - 1) / TPB), TPB, 0, c.stream>>>(row_of, col_idx, slot, nnzb, nbr, W, idxmap,
                                                                         bits);
  SP2_LAUNCH_CHECK();
}
void launch_popcount_rows(Ctx &c, const uint32_t *bits, int nbr, int W, int64_t *counts) {
  if (nbr <= 0) return;
  k_popcount_rows<<<nbr, TPB, 0, c.stream>>>(bits, nbr, W, counts);
  SP2_LAUNCH_CHECK();
}
void launch_extract_rows(Ctx &c, const uint32_t *bits, int nbr, int W, const int64_t *ptr, int32_t *cols,
                         int32_t *rows) {
  if (nbr <= 0) return;
  k_extract_rows<<<nbr, TPB, 0, c.stream>>>(bits, nbr, W, ptr, cols, rows);
  SP2_LAUNCH_CHECK();
}
void launch_symbolic(Ctx &c, const uint32_t *bits, const int64_t *adj_ptr, const int32_t *adj_col, int nbr, int W,
                     uint32_t *outbits, const uint32_t *bits2, const int64_t *adj_ptr2, const int32_t *adj_col2,
                     bool upper) {
  if (nbr <= 0) return;
  if (bits2 && !(adj_ptr2 && adj_col2)) fail(SP2_ERR_INVALID_ARG, "symbolic product: incomplete second operand");
  int WP = 1;
  while (WP < W && WP < TPB) WP <<= 1;
  k_symbolic<<<nbr, TPB, 0, c.stream>>>(bits, adj_ptr, adj_col, nbr, W, WP, outbits, bits2, adj_ptr2, adj_col2,
                                        upper);
  SP2_LAUNCH_CHECK();
}

void launch_or_upper(Ctx &c, const uint32_t *a, const uint32_t *b, int nbr, int W, uint32_t *out) {
  const int64_t n = (int64_t)nbr * W;
  if (n <= 0) return;
  k_or_upper<<<(unsigned)((n + TPB - 1) / TPB), TPB, 0, c.stream>>>(a, b, nbr, W, out);
  SP2_LAUNCH_CHECK();
}

void scan_exclusive_i64(Ctx &c, const int64_t *in, int64_t *out, int64_t n) {
  const int64_t ntiles = n > 0 ? (n + SCAN_TILE - 1) / SCAN_TILE : 0;
  Buf tsum = c.alloc(sizeof(int64_t) * (size_t)(ntiles + 1));
  if (ntiles > 0) {
    k_scan_tiles<<<(unsigned)ntiles, TPB, 0, c.stream>>>(in, n, tsum.as<int64_t>());
    SP2_LAUNCH_CHECK();
  }
  k_scan_top<<<1, TPB, 0, c.stream>>>(tsum.as<int64_t>(), ntiles, out + n);
  SP2_LAUNCH_CHECK();
  if (ntiles > 0) {
    k_scan_apply<<<(unsigned)ntiles, TPB, 0, c.stream>>>(in, n, tsum.as<int64_t>(), out);
    SP2_LAUNCH_CHECK();
  }
}

void launch_diag_missing(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t *counts) {
  k_diag_missing<<<grid_for(nbr), TPB, 0, c.stream>>>(row_ptr, col_idx, nbr, counts);
  SP2_LAUNCH_CHECK();
}
void launch_x0_pattern(Ctx &c, const int64_t *frow_ptr, const int32_t *fcol, int nbr, const int64_t *xrow_ptr,
                       int32_t *xcol, int32_t *src) {
  k_x0_pattern<<<grid_for(nbr), TPB, 0, c.stream>>>(frow_ptr, fcol, nbr, xrow_ptr, xcol, src);
  SP2_LAUNCH_CHECK();
}
void launch_init_x0(Ctx &c, const double *fval, const int32_t *src, const int32_t *xrow_of, const int32_t *xcol,
                    int64_t nnzb, int64_t n, double lmax, double w, double *xval) {
  if (nnzb <= 0) return;
  k_init_x0<<<(unsigned)nnzb, TPB, 0, c.stream>>>(fval, src, xrow_of, xcol, nnzb, n, lmax, w, xval);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
