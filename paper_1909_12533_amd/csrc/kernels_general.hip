// General (full-pattern) block storage: every present block of both
// triangles is stored as it is, the format of the general matrix wrapper of
// section "Implementation details" (section "Numerical experiments" compares
// it with the symmetric, upper-triangle one).  Pattern validation, block maps
// of a matrix or of its transpose, the union of an output bitmap with a
// second pattern and the diagonal, and the general form of a symmetric
// upper-BSR matrix.
#include "internal.h"

namespace sp2 {

namespace {

constexpr int TPB = 256;

// flag bit 1: column outside [0, nbr); bit 2: not strictly increasing;
// bit 4: row_ptr not monotone
__global__ void k_validate_general(const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb,
                                   int32_t *flag) {
  const int I = blockIdx.x;
  if (I >= nbr) return;
  const int64_t s = row_ptr[I], e = row_ptr[I + 1];
  if (threadIdx.x == 0 && (s > e || s < 0 || e > nnzb)) atomicOr(flag, 4);
  if (s > e || s < 0 || e > nnzb) return;
  for (int64_t b = s + threadIdx.x; b < e; b += blockDim.x) {
    const int32_t c = col_idx[b];
    if (c < 0 || c >= nbr) atomicOr(flag, 1);
    if (b > s && col_idx[b - 1] >= c) atomicOr(flag, 2);
  }
}

// one thread per stored block (I, J): entry (R, C) = (I, J), or (J, I) for
// the transpose, of the block map and the bitmaps
__global__ void k_build_maps_general(const int32_t *row_of, const int32_t *col_idx, const int32_t *slot,
                                     int64_t nnzb, int nbr, int W, bool transpose, int32_t *idxmap, uint32_t *bits) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int I = row_of[b], J = col_idx[b];
  const int R = transpose ? J : I, C = transpose ? I : J;
  if (idxmap) idxmap[(int64_t)R * nbr + C] = slot ? slot[b] : (int32_t)b;
  atomicOr(&bits[(int64_t)R * W + (C >> 5)], 1u << (C & 31));
}

__global__ void k_or_general(uint32_t *out, const uint32_t *g, int nbr, int W, bool diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)nbr * W) return;
  const int I = (int)(i / W), w = (int)(i % W);
  uint32_t v = out[i];
  if (g) v |= g[i];
  if (diag && (I >> 5) == w) v |= 1u << (I & 31);
  out[i] = v;
}

// one workgroup per output block: a copy of the stored block, or of its
// transpose through a padded LDS tile (reads and writes both row-major and
// coalesced)
__global__ __launch_bounds__(TPB) void k_expand_upper(const int32_t *row_of, const int32_t *col, int64_t nout,
                                                      int nbr, const int32_t *idxmap, const double *src,
                                                      double *dst) {
  __shared__ double tile[64][65];
  const int64_t o = blockIdx.x;
  if (o >= nout) return;
  const int I = row_of[o], J = col[o];
  const int32_t s = idxmap[(int64_t)I * nbr + J];
  const double *sb = src + (int64_t)s * BB;
  double *db = dst + o * BB;
  if (I <= J) {
    for (int e = threadIdx.x; e < BB; e += TPB) db[e] = sb[e];
    return;
  }
  for (int e = threadIdx.x; e < BB; e += TPB) tile[e >> 6][e & 63] = sb[e];
  __syncthreads();
  for (int e = threadIdx.x; e < BB; e += TPB) db[e] = tile[e & 63][e >> 6];
}

}  // namespace

void launch_validate_general(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb,
                             int32_t *flag) {
  if (nbr <= 0) return;
  k_validate_general<<<nbr, TPB, 0, c.stream>>>(row_ptr, col_idx, nbr, nnzb, flag);
  SP2_LAUNCH_CHECK();
}

void launch_build_maps_general(Ctx &c, const int32_t *row_of, const int32_t *col_idx, const int32_t *slot,
                               int64_t nnzb, int nbr, int W, bool transpose, int32_t *idxmap, uint32_t *bits) {
  if (idxmap) launch_fill_i32(c, idxmap, (int64_t)nbr * nbr, -1);
  launch_fill_u32(c, bits, (int64_t)nbr * W, 0u);
  if (nnzb <= 0) return;
  k_build_maps_general<<<(unsigned)((nnzb + TPB - 1) / TPB), TPB, 0, c.stream>>>(row_of, col_idx, slot, nnzb, nbr, W,
                                                                                 transpose, idxmap, bits);
  SP2_LAUNCH_CHECK();
}

void launch_or_general(Ctx &c, uint32_t *out, const uint32_t *g, int nbr, int W, bool diag) {
  const int64_t n = (int64_t)nbr * W;
  if (n <= 0 || (!g && !diag)) return;
  k_or_general<<<(unsigned)((n + TPB - 1) / TPB), TPB, 0, c.stream>>>(out, g, nbr, W, diag);
  SP2_LAUNCH_CHECK();
}

void launch_expand_upper(Ctx &c, const int32_t *row_of, const int32_t *col, int64_t nout, int nbr,
                         const int32_t *idxmap, const double *src, double *dst) {
  if (nout <= 0) return;
  k_expand_upper<<<(unsigned)nout, TPB, 0, c.stream>>>(row_of, col, nout, nbr, idxmap, src, dst);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
