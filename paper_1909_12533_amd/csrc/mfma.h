// Device building blocks shared by the MFMA kernels (gfx950): MFMA traits and
// accumulator layouts, 64 x 64 block staging through registers into padded
// LDS tiles, the wave-uniform K iterator over intersecting block-row
// bitmaps, and k-chunked fragment loads.
//
// MFMA 16x16x4 operand layout (f64 and f32): lane l holds A[l % 16][k(l / 16)]
// and B[k(l / 16)][l % 16] for the 4 k indices of the instruction; any
// assignment of k indices to lane groups works as long as A and B agree.  The
// accumulator element v of lane l is C[4 (l / 16) + v][l % 16] for f32, but
// C[4 v + l / 16][l % 16] for f64 (rows interleaved across the four result
// registers).
#pragma once

#include "internal.h"

namespace sp2 {
namespace dev {

constexpr int TPB = 256;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
template <> struct MF<double> {
  typedef d4 acc_t;
  static constexpr int LD = 66;  // padded LDS row (doubles): 16-byte aligned rows, spread banks
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // tile row of accumulator element v in lane group g = l / 16
  __device__ static inline int row(int g, int v) { return 4 * v + g; }
};
template <> struct MF<float> {
  typedef f4 acc_t;
  static constexpr int LD = 68;
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int g, int v) { return 4 * g + v; }
};

// a 64 x 64 block staged in registers: NCH 16-byte chunks per thread,
// chunk q = j * 256 + tid covers elements [q * EPC, (q + 1) * EPC)
template <typename T> struct Stage {
  static constexpr int EPC = 16 / sizeof(T);
  static constexpr int NCH = BB / EPC / TPB;
  uint4 r[NCH];
  __device__ inline void load(const T *blk) {
    const uint4 *p = reinterpret_cast<const uint4 *>(blk);
#pragma unroll
    for (int j = 0; j < NCH; ++j) r[j] = p[j * TPB + threadIdx.x];
  }
  __device__ inline void zero() {
#pragma unroll
    for (int j = 0; j < NCH; ++j) r[j] = make_uint4(0u, 0u, 0u, 0u);
  }
  __device__ inline void store(T *lds) const {
    constexpr int LD = MF<T>::LD;
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int e = (j * TPB + (int)threadIdx.x) * EPC;
      *reinterpret_cast<uint4 *>(lds + (e >> 6) * LD + (e & 63)) = r[j];
    }
  }
};

// wave-uniform iterator over the set bits of (ra & rb), i.e. the K with both
// X_IK and X_KJ stored
struct KIter {
  const uint32_t *ra, *rb;
  int W, wi;
  uint32_t m;
  __device__ inline int next() {
    while (m == 0) {
      ++wi;
      if (wi >= W) return -1;
      m = (uint32_t)__builtin_amdgcn_readfirstlane((int)(ra[wi] & rb[wi]));
    }
    const int bt = __builtin_ctz(m);
    m &= m - 1;
    return wi * 32 + bt;
  }
};

// one operand source: a value pool and its slot map
template <typename T> struct Src {
  const T *pool;
  const int32_t *idx;
};

// Fragments of one 16-deep k chunk for one wave: MFMA number s (0..3) of
// the chunk gives lane group g the k index k0 + 4 g + s, so a lane's four A
// values (and four B values) are contiguous along k; they are read with
// 16-byte LDS loads whenever the staged tile is contiguous along k.
template <typename T, bool TA, bool TB> struct Frag {
  T a[2][4], b[2][4];
  __device__ inline void load(const T *As, const T *Bs, int k0, int rowA, int colB) {
    constexpr int LD = MF<T>::LD;
    const int g = (threadIdx.x & 63) >> 4;
    const int kb = k0 + 4 * g;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int r = rowA + 16 * m;
      if (!TA) {  // A[r][k] = As[r][k], contiguous in k
        const T *p = As + r * LD + kb;
#pragma unroll
        for (int s = 0; s < 4; ++s) a[m][s] = p[s];
      } else {  // A[r][k] = As[k][r]
#pragma unroll
        for (int s = 0; s < 4; ++s) a[m][s] = As[(kb + s) * LD + r];
      }
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int c = colB + 16 * n;
      if (TB) {  // B[k][c] = Bs[c][k], contiguous in k
        const T *p = Bs + c * LD + kb;
#pragma unroll
        for (int s = 0; s < 4; ++s) b[n][s] = p[s];
      } else {  // B[k][c] = Bs[k][c]
#pragma unroll
        for (int s = 0; s < 4; ++s) b[n][s] = Bs[(kb + s) * LD + c];
      }
    }
  }
};

// one staged K block: 4 chunks of 16, next chunk's fragments loaded before
// the current chunk's MFMAs are issued
template <typename T, bool TA, bool TB>
__device__ inline void mma_block(typename MF<T>::acc_t (&acc)[2][2], const T *As, const T *Bs, int rowA, int colB) {
  Frag<T, TA, TB> f[2];
  f[0].load(As, Bs, 0, rowA, colB);
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    if (kc + 1 < 4) f[(kc + 1) & 1].load(As, Bs, 16 * (kc + 1), rowA, colB);
    const Frag<T, TA, TB> &cur = f[kc & 1];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[0][0] = MF<T>::op(cur.a[0][s], cur.b[0][s], acc[0][0]);
      acc[0][1] = MF<T>::op(cur.a[0][s], cur.b[1][s], acc[0][1]);
      acc[1][0] = MF<T>::op(cur.a[1][s], cur.b[0][s], acc[1][0]);
      acc[1][1] = MF<T>::op(cur.a[1][s], cur.b[1][s], acc[1][1]);
    }
  }
}

// accumulate sum_K A_IK B_KJ over K in bitsA[I] & bitsB[J], where A and B
// are symmetric matrices stored as upper blocks (A_IK for I > K is the
// transpose of stored (K, I))
template <typename T>
__device__ inline int accumulate(typename MF<T>::acc_t (&acc)[2][2], Src<T> A, const uint32_t *bitsA, Src<T> Bm,
                                 const uint32_t *bitsB, int I, int J, int nbr, int W, T *As, T *Bs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int rowA = 32 * wr + (lane & 15), colB = 32 * wc + (lane & 15);

  KIter it{bitsA + (int64_t)I * W, bitsB + (int64_t)J * W, W, -1, 0u};
  Stage<T> sa, sb;
  auto issue = [&](int K) -> bool {
    const int32_t pa = __builtin_amdgcn_readfirstlane(A.idx[(int64_t)I * nbr + K]);
    const int32_t pb = __builtin_amdgcn_readfirstlane(Bm.idx[(int64_t)K * nbr + J]);
    if (pa < 0 || pb < 0) {
      sa.zero();
      sb.zero();
      return false;
    }
    sa.load(A.pool + (int64_t)pa * BB);
    sb.load(Bm.pool + (int64_t)pb * BB);
    return true;
  };

  int nk = 0;
  int K = it.next();
  bool vcur = K >= 0 ? issue(K) : false;
  while (K >= 0) {
    const bool tA = I > K, tB = K > J;
    __syncthreads();  // every wave is done reading the previous tiles
    sa.store(As);
    sb.store(Bs);
    __syncthreads();
    const int Kn = it.next();
    const bool vn = Kn >= 0 ? issue(Kn) : false;  // next tiles in flight during the MFMAs
    if (vcur) {
      if (!tA && !tB)
        mma_block<T, false, false>(acc, As, Bs, rowA, colB);
      else if (!tA && tB)
        mma_block<T, false, true>(acc, As, Bs, rowA, colB);
      else if (tA && !tB)
        mma_block<T, true, false>(acc, As, Bs, rowA, colB);
      else
        mma_block<T, true, true>(acc, As, Bs, rowA, colB);
      ++nk;
    }
    K = Kn;
    vcur = vn;
  }
  return nk;
}


// XCD-aware tile index: workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), so XCD x runs workgroups x, x + 8, ...; giving
// it the contiguous chunk [x * chunk, (x + 1) * chunk) of the (super-tile
// ordered) tile list keeps tiles that share operand panels on the same L2.
// Returns -1 for the padding workgroups of the last chunk.
__device__ inline int64_t xcd_tile(const TileArgs &a) {
  const int64_t b = blockIdx.x;
  const int64_t t = (b % 8) * a.xcd_chunk + b / 8;
  return t < a.ntiles ? t : -1;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Epilogue of the square for the 64 x 64 output block (I, J) held by one wave
// in 4 x 4 MFMA 16 x 16 accumulator tiles: X_next = ca I + cb X + cc S is
// written at pattern position pos, and the block's partial sums (e^2 weighted
// by 2 off the diagonal, tr X, tr S, ||X_next||^2, #K) go to parts.
// rowf(g, v) is the tile row of accumulator element v of lane group g.
template <typename T, typename TO, typename ACC, typename RowF>
__device__ inline void square_epilogue(const ACC (&acc)[4][4], const TileArgs &a, int I, int J, int pos, const T *xp,
                                       int nk, RowF rowf) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int32_t sx = a.idxmap[(int64_t)I * a.nbr + J];
  const T *xb = sx >= 0 ? xp + (int64_t)sx * BB : nullptr;
  TO *ob = static_cast<TO *>(a.opool) + (int64_t)pos * BB;
  double e2 = 0.0, tx = 0.0, ts = 0.0, nr = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * m + rowf(g, q);
        const int c = 16 * n + l16;
        const double s = (double)acc[m][n][q];
        const double x = xb ? (double)xb[r * 64 + c] : 0.0;
        const bool dg = (I == J) && (r == c);
        const bool real_dg = dg && ((int64_t)I * B + r < a.n);
        const double o = a.cc * s + a.cb * x + (real_dg ? a.ca : 0.0);
        const TO ov = (TO)o;
        ob[r * 64 + c] = ov;
        const double od = (double)ov;
        nr += od * od;
        const double df = x - s;
        e2 += df * df;
        if (dg) {
          tx += x;
          ts += s;
        }
      }
  e2 = wave_sum(e2);
  tx = wave_sum(tx);
  ts = wave_sum(ts);
  nr = wave_sum(nr);
  if (lane == 0) {
    double *p = a.parts + (int64_t)pos * NPART;
    p[0] = (I == J) ? e2 : 2.0 * e2;
    p[1] = tx;
    p[2] = ts;
    p[3] = nr;
    p[4] = (double)nk;
  }
}

}  // namespace dev
}  // namespace sp2
