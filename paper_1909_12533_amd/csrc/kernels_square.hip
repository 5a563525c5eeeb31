// Anticommutator products on MFMA for the adjoint of the recursion:
// out = cb G + cc (G X + X G) on a given set of upper output blocks, with G
// and X symmetric block-sparse matrices stored as their upper triangles (a
// lower block is read as the transpose of its stored mirror by the fragment
// addressing).  This is the derivative of X -> a I + b X + c X^2 in the
// direction G (JVP) and, X being symmetric, also its adjoint applied to G
// (VJP).
//
// Work decomposition: one workgroup of 4 waves per output block (I, J); the
// two K loops run over the set bits of bitsG[I] & bitsX[J] and
// bitsX[I] & bitsG[J]; each K stages the two operand blocks through LDS
// (loaded one K ahead in registers) and each wave owns a 32 x 32 quadrant of
// the output as 2 x 2 tiles of 16 x 16 MFMA accumulators.
#include "mfma.h"

namespace sp2 {

namespace {

using namespace dev;

// out = cb G + cc (G X + X G) on the given output blocks (FP64), for the
// adjoint of X -> a I + b X + c X^2.
__global__ __launch_bounds__(TPB, 2) void k_anticommutator(AntiArgs a) {
  constexpr int LD = MF<double>::LD;
  __shared__ __align__(16) double As[64 * LD];
  __shared__ __align__(16) double Bs[64 * LD];
  const int64_t w = blockIdx.x;
  if (w >= a.nout) return;
  const int I = __builtin_amdgcn_readfirstlane(a.out_row[w]);
  const int J = __builtin_amdgcn_readfirstlane(a.out_col[w]);
  d4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[m][n] = d4{0, 0, 0, 0};
  const Src<double> G{a.gpool, a.gidxmap}, X{a.xpool, a.xidxmap};
  accumulate<double>(acc, G, a.gbits, X, a.xbits, I, J, a.nbr, a.W, As, Bs);
  accumulate<double>(acc, X, a.xbits, G, a.gbits, I, J, a.nbr, a.W, As, Bs);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, g = lane >> 4;
  const int32_t sg = a.gidxmap[(int64_t)I * a.nbr + J];
  const double *gb = sg >= 0 ? a.gpool + (int64_t)sg * BB : nullptr;
  double *ob = a.opool + w * BB;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 32 * wr + 16 * m + MF<double>::row(g, q);
        const int c = 32 * wc + 16 * n + l16;
        const double gv = gb ? gb[r * 64 + c] : 0.0;
        ob[r * 64 + c] = a.cc * acc[m][n][q] + a.cb * gv;
      }
}

}  // namespace

void launch_anticommutator(Ctx &c, const AntiArgs &a) {
  if (a.nout <= 0) return;
  k_anticommutator<<<(unsigned)a.nout, TPB, 0, c.stream>>>(a);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
