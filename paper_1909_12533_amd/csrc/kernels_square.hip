// Numeric block-sparse symmetric square on MFMA (gfx950), with the polynomial
// update, the idempotency error and the traces fused into its epilogue.
//
// Algorithm 2 needs, per iteration, the square S = X~_i^2: it gives both
// e_i = ||X~_i - X~_i^2||_F, t_i = tr(X~_i - X~_i^2) and the next iterate
// X_{i+1} = f_{i+1}(X~_i), which for both polynomial families is
// a I + b X~_i + c S:
//   p = 1: ((1 - alpha) I + alpha X)^2  -> (a, b, c) = ((1-alpha)^2, 2 alpha (1-alpha), alpha^2)
//   p = 0: 2 alpha X - (alpha X)^2      -> (a, b, c) = (0, 2 alpha, -alpha^2)
// Only upper blocks (I <= J) of S are formed (the symmetric wrapper of
// section "Implementation details").  A lower block X_KI (K > I) is read as
// the transpose of the stored X_IK: the transpose is folded into the LDS
// addressing of the MFMA operands, never materialised.
//
// Work decomposition: one workgroup of 4 waves per output block (I, J); the
// K loop runs over the set bits of bits[I] & bits[J] (block rows I and J of
// the symmetric pattern), so no triple list is ever stored.  Each K stages
// X_IK and X_KJ (64 x 64 each) through LDS, loaded with 16-byte coalesced
// global reads one K ahead in registers; each wave owns a 32 x 32 quadrant
// of the output as 2 x 2 tiles of 16 x 16 MFMA accumulators.
//
// MFMA 16x16x4 operand layout used here (f64 and f32): lane l holds
// A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16].  The accumulator element
// v of lane l is C[4 (l / 16) + v][l % 16] for f32, but C[4 v + l / 16][l % 16]
// for f64 (rows interleaved across the four result registers).
#include "internal.h"

namespace sp2 {

namespace {

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

// accumulate sum_K A_IK B_KJ over K in bitsA[I] & bitsB[J], where A and B
// are symmetric matrices stored as upper blocks (A_IK for I > K is the
// transpose of stored (K, I))
template <typename T>
__device__ inline int accumulate(typename MF<T>::acc_t (&acc)[2][2], Src<T> A, const uint32_t *bitsA, Src<T> Bm,
                                 const uint32_t *bitsB, int I, int J, int nbr, int W, T *As, T *Bs) {
  constexpr int LD = MF<T>::LD;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, g = lane >> 4;

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
      // A[r][k] = tA ? As[k][r] : As[r][k];  B[k][c] = tB ? Bs[c][k] : Bs[k][c]
      const int sAr = tA ? 1 : LD, sAk = tA ? LD : 1;
      const int sBk = tB ? 1 : LD, sBc = tB ? LD : 1;
      const T *pa = As + (32 * wr + l16) * sAr + g * sAk;
      const T *pb = Bs + g * sBk + (32 * wc + l16) * sBc;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int ka = 4 * s * sAk, kb = 4 * s * sBk;
        const T a0 = pa[ka], a1 = pa[16 * sAr + ka];
        const T b0 = pb[kb], b1 = pb[kb + 16 * sBc];
        acc[0][0] = MF<T>::op(a0, b0, acc[0][0]);
        acc[0][1] = MF<T>::op(a0, b1, acc[0][1]);
        acc[1][0] = MF<T>::op(a1, b0, acc[1][0]);
        acc[1][1] = MF<T>::op(a1, b1, acc[1][1]);
      }
      ++nk;
    }
    K = Kn;
    vcur = vn;
  }
  return nk;
}

// deterministic workgroup sum of 4 values (fixed butterfly + fixed wave order)
__device__ inline void wg_sum4(double (&v)[4], double (&out)[4]) {
  __shared__ double red[TPB / 64][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int j = 0; j < 4; ++j) red[wave][j] = v[j];
  __syncthreads();
  for (int j = 0; j < 4; ++j) out[j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
}

template <typename T, typename TO>
__global__ __launch_bounds__(TPB, 2) void k_square(SquareArgs a) {
  constexpr int LD = MF<T>::LD;
  __shared__ __align__(16) T As[64 * LD];
  __shared__ __align__(16) T Bs[64 * LD];
  const int64_t w = blockIdx.x;
  if (w >= a.nout) return;
  const int I = __builtin_amdgcn_readfirstlane(a.out_row[w]);
  const int J = __builtin_amdgcn_readfirstlane(a.out_col[w]);
  const T *xp = static_cast<const T *>(a.xpool);

  typename MF<T>::acc_t acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[m][n] = typename MF<T>::acc_t{0, 0, 0, 0};

  const Src<T> X{xp, a.idxmap};
  const int nk = accumulate<T>(acc, X, a.bits, X, a.bits, I, J, a.nbr, a.W, As, Bs);

  // epilogue: X_next = ca I + cb X + cc S, partial sums of e^2, traces, norm
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, g = lane >> 4;
  const int32_t sx = a.idxmap[(int64_t)I * a.nbr + J];
  const T *xb = sx >= 0 ? xp + (int64_t)sx * BB : nullptr;
  TO *ob = static_cast<TO *>(a.opool) + w * BB;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // e2, trX, trS, nrm2
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 32 * wr + 16 * m + MF<T>::row(g, q);
        const int c = 32 * wc + 16 * n + l16;
        const double s = (double)acc[m][n][q];
        const double x = xb ? (double)xb[r * 64 + c] : 0.0;
        const bool dg = (I == J) && (r == c);
        const bool real_dg = dg && ((int64_t)I * B + r < a.n);
        const double o = a.cc * s + a.cb * x + (real_dg ? a.ca : 0.0);
        const TO ov = (TO)o;
        ob[r * 64 + c] = ov;
        const double od = (double)ov;
        v[3] += od * od;
        const double df = x - s;
        v[0] += df * df;
        if (dg) {
          v[1] += x;
          v[2] += s;
        }
      }
  double tot[4];
  wg_sum4(v, tot);
  if (threadIdx.x == 0) {
    double *p = a.parts + w * NPART;
    p[0] = (I == J) ? tot[0] : 2.0 * tot[0];
    p[1] = tot[1];
    p[2] = tot[2];
    p[3] = tot[3];
    p[4] = (double)nk;
  }
}

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

void launch_square(Ctx &c, int mode, const SquareArgs &a) {
  if (a.nout <= 0) return;
  const unsigned g = (unsigned)a.nout;
  if (mode == M_F64) {
    if (a.xprec != P64 || a.oprec != P64) fail(SP2_ERR_INVALID_ARG, "FP64 square needs FP64 pools");
    k_square<double, double><<<g, TPB, 0, c.stream>>>(a);
  } else if (mode == M_F32) {
    if (a.xprec != P32) fail(SP2_ERR_INVALID_ARG, "FP32 square needs an FP32 input pool");
    if (a.oprec == P32)
      k_square<float, float><<<g, TPB, 0, c.stream>>>(a);
    else
      k_square<float, double><<<g, TPB, 0, c.stream>>>(a);
  } else {
    fail(SP2_ERR_INVALID_ARG, "square mode not available");
  }
  SP2_LAUNCH_CHECK();
}

void launch_anticommutator(Ctx &c, const AntiArgs &a) {
  if (a.nout <= 0) return;
  k_anticommutator<<<(unsigned)a.nout, TPB, 0, c.stream>>>(a);
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
