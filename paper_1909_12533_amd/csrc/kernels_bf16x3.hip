// BF16x3 split-precision variant of the tiled square (low-precision phase of
// the mixed-precision policy): every FP32 operand value x is split into
// hi = bf16(x) and lo = bf16(x - hi) (round to nearest even; x - hi is exact in
// FP32), and each block product is hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the dropped lo*lo term and
// the residual x - hi - lo are both of relative size ~2^-16).
//
// Same work decomposition as k_square_tile (one workgroup per 2 x 2 output
// tile, one 64 x 64 output block per wave).  The split happens once per
// element while staging: the four operand blocks of a K are loaded as FP32,
// split in registers and written to LDS as two bf16 planes each, always
// k-contiguous (A as [row][k], B as [column][k]) so that every MFMA operand
// (8 consecutive k of one row/column) is a single 16-byte LDS read.  Operands
// whose k index runs along the stored rows are loaded as 4-row column chunks
// (4-byte loads, coalesced along the column index) so that their transposed
// LDS write is still one 8-byte store per plane.
#include "mfma.h"

namespace sp2 {

namespace {

using namespace dev;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int LDH = 72;           // bf16 per plane row (64 + 8 pad): 144-byte rows
constexpr int PLANE = 64 * LDH;   // bf16 per plane

__device__ inline uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// split four FP32 values into packed bf16 hi and lo pairs
__device__ inline void split4(u32x4 v, u32x2 &hi, u32x2 &lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float x = __uint_as_float(v[j]);
    h[j] = bf16_rne(x);
    l[j] = bf16_rne(x - __uint_as_float(h[j] << 16));
  }
  hi = u32x2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
  lo = u32x2{l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
}

__device__ inline f4 mfma_bf16(u32x4 a, u32x4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

template <typename TO, bool GEN>
__global__ __launch_bounds__(TPB, 1) void k_square_tile_bf16x3(TileArgs a) {
  // operand o (A0, A1, B0, B1) x plane (hi, lo)
  __shared__ __align__(16) uint16_t L[4][2][PLANE];
  const int64_t t = xcd_tile(a);
  if (t < 0) return;
  const int nbr = a.nbr, W = a.W;
  const int I0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t]);
  const int J0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t + 1]);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ia = wave >> 1, jb = wave & 1;
  const int I = I0 + ia, J = J0 + jb;
  const bool has_i1 = I0 + 1 < nbr, has_j1 = J0 + 1 < nbr;
  int32_t pos = -1;
  if (I < nbr && J < nbr && I <= J) pos = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + J]);
  const float *xp = static_cast<const float *>(a.xpool);
  const float *yp = static_cast<const float *>(GEN ? a.ypool : a.xpool);

  f4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = f4{0, 0, 0, 0};

  // K scan as in the FP64 / FP32 kernel (second pass: operands swapped)
  const uint32_t *ybits = GEN ? a.ybits : a.bits;
  const uint32_t *bI0 = a.bits + (int64_t)I0 * W, *bI1 = a.bits + (int64_t)(has_i1 ? I0 + 1 : I0) * W;
  const uint32_t *bJ0 = ybits + (int64_t)J0 * W, *bJ1 = ybits + (int64_t)(has_j1 ? J0 + 1 : J0) * W;
  int wi = -1, pass = 0, kpass = 0;
  uint32_t mask = 0u;
  auto next_k = [&]() -> int {
    while (mask == 0u) {
      ++wi;
      if (wi >= W) {
        if (!GEN || pass + 1 >= a.npass) return -1;
        ++pass;
        wi = -1;
        bI0 = a.ybits + (int64_t)I0 * W;
        bI1 = a.ybits + (int64_t)(has_i1 ? I0 + 1 : I0) * W;
        bJ0 = a.bits + (int64_t)J0 * W;
        bJ1 = a.bits + (int64_t)(has_j1 ? J0 + 1 : J0) * W;
        continue;
      }
      const uint32_t ra = bI0[wi] | (has_i1 ? bI1[wi] : 0u);
      const uint32_t rb = bJ0[wi] | (has_j1 ? bJ1[wi] : 0u);
      mask = (uint32_t)__builtin_amdgcn_readfirstlane((int)(ra & rb));
    }
    kpass = pass;
    const int K = wi * 32 + __builtin_ctz(mask);
    mask &= mask - 1u;
    return K;
  };

  // staged FP32 values of the four operands, 16 per thread each
  u32x4 r0[4], r1[4], r2[4], r3[4];
  int32_t s0 = -1, s1 = -1, s2 = -1, s3 = -1;
  bool k0 = true, k1 = true, k2 = true, k3 = true;  // k runs along the stored columns
  const float *p0 = xp, *p1 = xp, *p2 = yp, *p3 = yp;  // source pools of the staged blocks
  uint32_t g0 = 0u, g1 = 0u, g2 = 0u, g3 = 0u;         // sign bit to flip per staged block
  constexpr uint32_t SGN = 0x80000000u;
  const int cc = tid & 63, rg = tid >> 6;
// row chunks (k along stored columns): 16-byte loads; column chunks: rows 16 rg + 4 jj + j of column cc
#define SP2_LOAD(R, P, SL, KCOL)                                                                   \
  do {                                                                                             \
    if ((SL) >= 0) {                                                                               \
      const float *blk_ = (P) + (int64_t)(SL) * BB;                                                \
      if (KCOL) {                                                                                  \
        const u32x4 *p_ = reinterpret_cast<const u32x4 *>(blk_) + tid;                             \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) R[j] = p_[j * TPB];                          \
      } else {                                                                                     \
        const uint32_t *p_ = reinterpret_cast<const uint32_t *>(blk_) + cc;                        \
        _Pragma("unroll") for (int jj = 0; jj < 4; ++jj) {                                         \
          const int r_ = 16 * rg + 4 * jj;                                                         \
          R[jj] = u32x4{p_[(r_ + 0) * 64], p_[(r_ + 1) * 64], p_[(r_ + 2) * 64], p_[(r_ + 3) * 64]}; \
        }                                                                                          \
      }                                                                                            \
    }                                                                                              \
  } while (0)
#define SP2_ISSUE(KK, KP)                                                                  \
  do {                                                                                     \
    const int32_t *li_ = (GEN && (KP)) ? a.yidxmap : a.idxmap;                             \
    const int32_t *ri_ = GEN ? ((KP) ? a.idxmap : a.yidxmap) : a.idxmap;                   \
    p0 = p1 = (GEN && (KP)) ? yp : xp;                                                     \
    p2 = p3 = (GEN && (KP)) ? xp : yp;                                                     \
    s0 = __builtin_amdgcn_readfirstlane(li_[(int64_t)I0 * nbr + (KK)]);                    \
    s1 = has_i1 ? __builtin_amdgcn_readfirstlane(li_[(int64_t)(I0 + 1) * nbr + (KK)]) : -1; \
    s2 = __builtin_amdgcn_readfirstlane(ri_[(int64_t)(KK) * nbr + J0]);                    \
    s3 = has_j1 ? __builtin_amdgcn_readfirstlane(ri_[(int64_t)(KK) * nbr + J0 + 1]) : -1;  \
    k0 = I0 <= (KK);                                                                       \
    k1 = I0 + 1 <= (KK);                                                                   \
    k2 = (KK) > J0;                                                                        \
    k3 = (KK) > J0 + 1;                                                                    \
    if (GEN) {                                                                             \
      const bool la_ = (KP) ? a.yanti : a.xanti, ra_ = (KP) ? a.xanti : a.yanti;           \
      const bool ng_ = (KP) && a.neg2;                                                     \
      g0 = ((la_ && !k0) != ng_) ? SGN : 0u;                                               \
      g1 = ((la_ && !k1) != ng_) ? SGN : 0u;                                               \
      g2 = (ra_ && k2) ? SGN : 0u;                                                         \
      g3 = (ra_ && k3) ? SGN : 0u;                                                         \
    }                                                                                      \
    SP2_LOAD(r0, p0, s0, k0);                                                              \
    SP2_LOAD(r1, p1, s1, k1);                                                              \
    SP2_LOAD(r2, p2, s2, k2);                                                              \
    SP2_LOAD(r3, p3, s3, k3);                                                              \
  } while (0)
// split and write one operand into its two planes, k-contiguous
#define SP2_STORE(R, SL, KCOL, O, G)                                                              \
  do {                                                                                            \
    if ((SL) >= 0) {                                                                              \
      uint16_t *ph_ = L[O][0], *pl_ = L[O][1];                                                    \
      _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                             \
        u32x2 hi_, lo_;                                                                           \
        split4(GEN ? (R[j] ^ u32x4{(G), (G), (G), (G)}) : R[j], hi_, lo_);                        \
        int off_;                                                                                 \
        if (KCOL) {                                                                               \
          const int e_ = (j * TPB + tid) * 4;                                                     \
          off_ = (e_ >> 6) * LDH + (e_ & 63);                                                     \
        } else {                                                                                  \
          off_ = cc * LDH + 16 * rg + 4 * j;                                                      \
        }                                                                                         \
        *reinterpret_cast<u32x2 *>(ph_ + off_) = hi_;                                             \
        *reinterpret_cast<u32x2 *>(pl_ + off_) = lo_;                                             \
      }                                                                                           \
    }                                                                                             \
  } while (0)

  const int l16 = lane & 15, g = lane >> 4;
  int nk = 0;
  int K = next_k();
  if (K >= 0) SP2_ISSUE(K, kpass);
  while (K >= 0) {
    const int32_t c0 = s0, c1 = s1, c2 = s2, c3 = s3;
    __syncthreads();  // previous planes fully consumed
    SP2_STORE(r0, c0, k0, 0, g0);
    SP2_STORE(r1, c1, k1, 1, g1);
    SP2_STORE(r2, c2, k2, 2, g2);
    SP2_STORE(r3, c3, k3, 3, g3);
    __syncthreads();
    const int Kn = next_k();
    if (Kn >= 0) SP2_ISSUE(Kn, kpass);  // next K's blocks in flight during the MFMAs
    const int32_t sa = ia ? c1 : c0, sb = jb ? c3 : c2;
    if (pos >= 0 && sa >= 0 && sb >= 0) {
      const uint16_t *ah = L[ia][0], *al = L[ia][1], *bh = L[2 + jb][0], *bl = L[2 + jb][1];
#pragma unroll
      for (int ks = 0; ks < 64; ks += 32) {
        u32x4 fah[4], fal[4], fbh[4], fbl[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int o = (16 * m + l16) * LDH + ks + 8 * g;
          fah[m] = *reinterpret_cast<const u32x4 *>(ah + o);
          fal[m] = *reinterpret_cast<const u32x4 *>(al + o);
          fbh[m] = *reinterpret_cast<const u32x4 *>(bh + o);
          fbl[m] = *reinterpret_cast<const u32x4 *>(bl + o);
        }
        // small products first, each accumulator touched once per sweep
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fal[m], fbh[n], acc[m][n]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fah[m], fbl[n], acc[m][n]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fah[m], fbh[n], acc[m][n]);
      }
      ++nk;
    }
    K = Kn;
  }
#undef SP2_ISSUE
#undef SP2_LOAD
#undef SP2_STORE
  if (pos < 0) return;
  // f32 16 x 16 accumulator layout: element v of lane group g is row 4 g + v
  square_epilogue<float, TO>(acc, a, I, J, pos, nk, [](int gg, int q) { return 4 * gg + q; });
}

}  // namespace

void launch_square_tile_bf16x3(Ctx &c, const TileArgs &a) {
  if (a.ntiles <= 0) return;
  if (a.xprec != P32) fail(SP2_ERR_INVALID_ARG, "BF16x3 square needs an FP32 input pool");
  const bool gen = a.ypool != a.xpool || a.npass != 1 || a.xanti || a.yanti;
  const unsigned g = (unsigned)(8 * a.xcd_chunk);
  if (a.oprec == P32) {
    if (gen)
      k_square_tile_bf16x3<float, true><<<g, TPB, 0, c.stream>>>(a);
    else
      k_square_tile_bf16x3<float, false><<<g, TPB, 0, c.stream>>>(a);
  } else {
    if (gen)
      k_square_tile_bf16x3<double, true><<<g, TPB, 0, c.stream>>>(a);
    else
      k_square_tile_bf16x3<double, false><<<g, TPB, 0, c.stream>>>(a);
  }
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
