// Device building blocks shared by the MFMA kernels (gfx950): MFMA traits and
// accumulator layouts, the staging geometry of 64 x 64 blocks, the
// XCD-aware tile order, wave reductions and the fused epilogue.
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

// staging of a 64 x 64 block through registers: NCH 16-byte chunks per
// thread, chunk q = j * 256 + tid covers elements [q * EPC, (q + 1) * EPC)
template <typename T> struct Stage {
  static constexpr int EPC = 16 / sizeof(T);
  static constexpr int NCH = BB / EPC / TPB;
};

// XCD-aware tile index: workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), so XCD x runs workgroups x, x + 8, ...; giving
// it the contiguous chunk [x * chunk, (x + 1) * chunk) of the (super-tile
// ordered) tile list keeps tiles that share operand panels on the same L2.
// Returns -1 for the padding workgroups of the last chunk.
#ifndef SP2_XCD_MAP
#define SP2_XCD_MAP 1
#endif
__device__ inline int64_t xcd_tile(const TileArgs &a) {
  const int64_t b = blockIdx.x;
  const int64_t t = SP2_XCD_MAP ? (b % 8) * a.xcd_chunk + b / 8 : b;
  return t < a.ntiles ? t : -1;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Epilogue for the rows r0 + 16 m + rowf(g, v) (m < MT) of the 64 x 64 output
// block (I, J), held by one wave in MT x 4 MFMA 16 x 16 accumulator tiles S:
// out = ca I + cb G + cc S is written at pattern position pos, and the
// wave's partial sums (||G - S||^2 weighted by 2 off the diagonal unless the
// storage is general, tr G, tr S,
// ||out||^2) are returned, reduced over the wave.  In the square G = X, so
// these are e^2, tr X~ and tr X~^2.
struct EpiSums {
  double e2, tx, ts, nr;
};

template <typename T, typename TO, int MT, typename ACC, typename RowF>
__device__ inline EpiSums epilogue_rows(const ACC (&acc)[MT][4], const TileArgs &a, int I, int J, int pos, int r0,
                                        RowF rowf) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int32_t sx = a.gpool ? a.gidxmap[(int64_t)I * a.nbr + J] : -1;
  const T *xb = sx >= 0 ? static_cast<const T *>(a.gpool) + (int64_t)sx * BB : nullptr;
  TO *ob = static_cast<TO *>(a.opool) + (int64_t)pos * BB;
  double e2 = 0.0, tx = 0.0, ts = 0.0, nr = 0.0;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + 16 * m + rowf(g, q);
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
  EpiSums ps;
  ps.e2 = wave_sum((I == J || a.full) ? e2 : 2.0 * e2);
  ps.tx = wave_sum(tx);
  ps.ts = wave_sum(ts);
  ps.nr = wave_sum(nr);
  return ps;
}

// the whole block in one wave (4 x 4 tiles): write the block's parts {e^2, tr G,
// tr S, ||out||^2, #K}
template <typename T, typename TO, typename ACC, typename RowF>
__device__ inline void square_epilogue(const ACC (&acc)[4][4], const TileArgs &a, int I, int J, int pos, int nk,
                                       RowF rowf) {
  const EpiSums ps = epilogue_rows<T, TO, 4>(acc, a, I, J, pos, 0, rowf);
  if ((threadIdx.x & 63) == 0) {
    double *p = a.parts + (int64_t)pos * NPART;
    p[0] = ps.e2;
    p[1] = ps.tx;
    p[2] = ps.ts;
    p[3] = ps.nr;
    p[4] = (double)nk;
  }
}

}  // namespace dev
}  // namespace sp2
