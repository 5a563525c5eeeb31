// BF16x3 split-precision variant of the tiled square (low-precision phase of
// the mixed-precision policy): every FP32 operand value x is split into
// hi = bf16(x) and lo = bf16(x - hi) (round to nearest even; x - hi is exact in
// FP32), and each block product is hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the dropped lo*lo term and
// the residual x - hi - lo are both of relative size ~2^-16).
//
// The split is done once per operand matrix by k_pack_bf16x3, which writes
// every stored block S as four bf16 planes: N = S (row-major) and T = S^T,
// each as hi and lo.  An MFMA operand wants 8 consecutive k of one row (A) or
// one column (B) in a single 16-byte LDS read, i.e. k-contiguous rows:
//   A = X_{I,K}: rows of S = X_IK (image N) when I <= K, of S = X_KI^T
//                (image T) when I > K;
//   B = X_{K,J}: stored as [column][k]: image T of S = X_KJ when K <= J,
//                image N of S = X_JK when K > J.
// So every staging load is a contiguous 16 KB copy (hi and lo planes of one
// image) and the tile kernel does no conversion arithmetic.
//
// Same work decomposition as k_square_tile (one workgroup per 2 x 2 output
// tile, one 64 x 64 output block per wave); the workgroup needs 72 KB of LDS
// and at most 256 registers per lane, so two workgroups share a CU and one's
// staging overlaps the other's MFMAs.
#include "mfma.h"

namespace sp2 {

namespace {

using namespace dev;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int LDH = 72;            // bf16 per LDS plane row (64 + 8 pad): 144-byte rows
constexpr int PLANE = 64 * LDH;    // bf16 per LDS plane
constexpr int IMG_Q = 1024;        // 16-byte chunks per image (hi + lo planes, 2 x 8 KB)
constexpr int BLK_Q = 2 * IMG_Q;   // 16-byte chunks per packed block (images N, T)

__device__ inline uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ inline f4 mfma_bf16(u32x4 a, u32x4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// One workgroup per stored block b: packed[slot] = N_hi, N_lo, T_hi, T_lo
// (4096 bf16 each).  The block goes through LDS so that both images are
// written with consecutive threads on consecutive elements.
__global__ __launch_bounds__(TPB) void k_pack_bf16x3(const float *pool, const int32_t *slot, int64_t nblocks,
                                                     uint16_t *packed) {
  __shared__ float t[64][65];
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t s = slot ? slot[b] : b;
  const float *src = pool + s * BB;
  for (int e = threadIdx.x; e < BB; e += TPB) t[e >> 6][e & 63] = src[e];
  __syncthreads();
  uint16_t *dst = packed + s * (int64_t)(4 * BB);
  for (int e = threadIdx.x; e < BB; e += TPB) {
    const int r = e >> 6, c = e & 63;
    const float xn = t[r][c], xt = t[c][r];
    const uint32_t hn = bf16_rne(xn), ht = bf16_rne(xt);
    dst[e] = (uint16_t)hn;
    dst[BB + e] = (uint16_t)bf16_rne(xn - __uint_as_float(hn << 16));
    dst[2 * BB + e] = (uint16_t)ht;
    dst[3 * BB + e] = (uint16_t)bf16_rne(xt - __uint_as_float(ht << 16));
  }
}

// FULL (with GEN, one pass): general storage, A = X_{I,K} always image N of
// its stored block, B = Y_{K,J} always image T; output blocks of both triangles
template <typename TO, bool GEN, bool FULL = false>
__global__ __launch_bounds__(TPB, 2) void k_square_tile_bf16x3(TileArgs a) {
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
  if (I < nbr && J < nbr && (FULL || I <= J)) pos = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + J]);
  const u32x4 *xq = static_cast<const u32x4 *>(a.xpack);
  const u32x4 *yq = static_cast<const u32x4 *>(GEN ? a.ypack : a.xpack);

  f4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = f4{0, 0, 0, 0};

  // K scan as in the FP64 / FP32 kernel (second pass: operands swapped).  The
  // slot maps are symmetric (both orientations of a stored block hold its slot),
  // so the right operand's slots are read along row J of the map: consecutive
  // K share scalar cache lines.
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

  // staged images of the four operands, 4 chunks of 16 bytes per thread each
  u32x4 r0[4], r1[4], r2[4], r3[4];
  int32_t s0 = -1, s1 = -1, s2 = -1, s3 = -1;
  uint32_t g0 = 0u, g1 = 0u, g2 = 0u, g3 = 0u;  // 0x80008000 to negate a staged block
  constexpr uint32_t SGN2 = 0x80008000u;
// image N (NIMG) or T of the block in slot SL; chunk j * 256 + tid of the
// image.  An absent block (SL < 0) stages zeros: the staging registers are then
// written on every path, so the loads of the four operands are issued back to
// back with no wait on the previous step's loads between them.
#define SP2_LOAD(R, Q, SL, NIMG)                                                    \
  do {                                                                              \
    if ((SL) >= 0) {                                                                \
      const u32x4 *img_ = (Q) + (int64_t)(SL) * BLK_Q + ((NIMG) ? 0 : IMG_Q) + tid; \
      _Pragma("unroll") for (int j = 0; j < 4; ++j) R[j] = img_[j * TPB];           \
    } else {                                                                        \
      _Pragma("unroll") for (int j = 0; j < 4; ++j) R[j] = u32x4{0u, 0u, 0u, 0u};   \
    }                                                                               \
  } while (0)
#define SP2_ISSUE(KK, KP)                                                                    \
  do {                                                                                       \
    const int32_t *li_ = (GEN && (KP)) ? a.yidxmap : a.idxmap;                               \
    const int32_t *ri_ = GEN ? ((KP) ? a.idxmap : a.yidxmap) : a.idxmap;                     \
    const u32x4 *lq_ = (GEN && (KP)) ? yq : xq, *rq_ = (GEN && (KP)) ? xq : yq;              \
    s0 = __builtin_amdgcn_readfirstlane(li_[(int64_t)I0 * nbr + (KK)]);                      \
    s1 = has_i1 ? __builtin_amdgcn_readfirstlane(li_[(int64_t)(I0 + 1) * nbr + (KK)]) : -1;   \
    s2 = __builtin_amdgcn_readfirstlane(ri_[(int64_t)J0 * nbr + (KK)]);                      \
    s3 = has_j1 ? __builtin_amdgcn_readfirstlane(ri_[(int64_t)(J0 + 1) * nbr + (KK)]) : -1;  \
    const bool n0_ = FULL || I0 <= (KK), n1_ = FULL || I0 + 1 <= (KK);                       \
    const bool n2_ = !FULL && (KK) > J0, n3_ = !FULL && (KK) > J0 + 1;                       \
    if (GEN) {                                                                               \
      const bool la_ = (KP) ? a.yanti : a.xanti, ra_ = (KP) ? a.xanti : a.yanti;             \
      const bool ng_ = (KP) && a.neg2;                                                       \
      g0 = ((la_ && !n0_) != ng_) ? SGN2 : 0u;                                               \
      g1 = ((la_ && !n1_) != ng_) ? SGN2 : 0u;                                               \
      g2 = (ra_ && n2_) ? SGN2 : 0u;                                                         \
      g3 = (ra_ && n3_) ? SGN2 : 0u;                                                         \
    }                                                                                        \
    SP2_LOAD(r0, lq_, s0, n0_);                                                              \
    SP2_LOAD(r1, lq_, s1, n1_);                                                              \
    SP2_LOAD(r2, rq_, s2, n2_);                                                              \
    SP2_LOAD(r3, rq_, s3, n3_);                                                              \
  } while (0)
// chunk j * 256 + tid: plane j / 2, row ((j & 1) * 256 + tid) / 8, 16-byte column chunk tid % 8
#define SP2_STORE(R, O, G)                                                             \
  do {                                                                                 \
    _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                    \
      const int pq_ = ((j & 1) << 8) + tid;                                            \
      uint16_t *d_ = &L[O][j >> 1][(pq_ >> 3) * LDH + (pq_ & 7) * 8];                   \
      *reinterpret_cast<u32x4 *>(d_) = GEN ? (R[j] ^ u32x4{(G), (G), (G), (G)}) : R[j]; \
    }                                                                                  \
  } while (0)

  const int l16 = lane & 15, g = lane >> 4;
  int nk = 0;
  int K = next_k();
  if (K >= 0) SP2_ISSUE(K, kpass);
  while (K >= 0) {
    const int32_t c0 = s0, c1 = s1, c2 = s2, c3 = s3;
    __syncthreads();  // previous planes fully consumed
    SP2_STORE(r0, 0, g0);
    SP2_STORE(r1, 1, g1);
    SP2_STORE(r2, 2, g2);
    SP2_STORE(r3, 3, g3);
    __syncthreads();
    const int Kn = next_k();
    if (Kn >= 0) SP2_ISSUE(Kn, kpass);  // next K's images in flight during the MFMAs
    const int32_t sa = ia ? c1 : c0, sb = jb ? c3 : c2;
    if (pos >= 0 && sa >= 0 && sb >= 0) {
      const uint16_t *ah = L[ia][0], *al = L[ia][1], *bh = L[2 + jb][0], *bl = L[2 + jb][1];
#pragma unroll
      for (int ks = 0; ks < 64; ks += 32) {
        u32x4 fbh[4], fbl[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int o = (16 * n + l16) * LDH + ks + 8 * g;
          fbh[n] = *reinterpret_cast<const u32x4 *>(bh + o);
          fbl[n] = *reinterpret_cast<const u32x4 *>(bl + o);
        }
        // per A tile: the four accumulators of its row take lo*hi, then
        // hi*hi, then hi*lo (four independent MFMAs between dependent ones)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int o = (16 * m + l16) * LDH + ks + 8 * g;
          const u32x4 fah = *reinterpret_cast<const u32x4 *>(ah + o);
          const u32x4 fal = *reinterpret_cast<const u32x4 *>(al + o);
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fal, fbh[n], acc[m][n]);
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fah, fbh[n], acc[m][n]);
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n] = mfma_bf16(fah, fbl[n], acc[m][n]);
        }
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

// ---------------------------------------------------------------------------
// 4 x 4 tiles of output blocks, for dense patterns.  The k_square_tile_bf16x3
// above is bound by operand traffic: each staged block serves two products.
// Here the workgroup stages the images of four left operand blocks (rows
// I0..I0+3 at K) and four right ones (columns J0..J0+3) for 16 products, half
// the traffic per product.  The images go straight from global memory to LDS
// (global_load_lds_dwordx4), one 32-deep k half at a time, double-buffered:
// k half 0 of every K lives in stage S0 and k half 1 in S1, so the load of
// the next half overlaps the MFMAs of the current one, and no registers are
// spent on staging.  8 waves, two per SIMD; wave w multiplies row block
// I0 + w / 2 by column blocks J0 + 2 (w % 2) + b, b = 0, 1 (2 x 16
// accumulator tiles).  Accumulation order per output element is that of
// k_square_tile_bf16x3 (K ascending; k half 0 then 1; lo*hi, hi*hi, hi*lo),
// so the two kernels give bit-identical results.
//
// LDS layout of one operand plane in a stage: 64 rows x 32 bf16 (64 bytes,
// four 16-byte chunks); logical chunk g of row R sits at chunk g ^ swz(R),
// swz(R) = bit2(R) | (bit1(R) ^ bit3(R)) << 1, which makes the 16-byte
// fragment reads of 16 (or 8) consecutive rows hit distinct banks.  A wave's
// load instruction writes 1 KB contiguously (lane l at byte 16 l), i.e.
// 16 rows; each lane fetches the global chunk that belongs at its slot.

__device__ inline int swz(int R) { return ((R >> 2) & 1) | ((((R >> 1) ^ (R >> 3)) & 1) << 1); }

constexpr int HPLANE = 64 * 32;  // bf16 per operand plane and k half

// a staged K, as one wave sees it: the slots (-1: absent) and sign masks of
// the operand blocks it multiplies (row ia, columns jp and jp + 1), and the
// slot of the operand it loads into LDS (operand w: A0..A3 = rows I0..I0+3 at
// K, B0..B3 = columns J0..J0+3)
struct Stage4 {
  int K, kp;
  int32_t sa, sb0, sb1, sd;
  uint32_t ga, gb0, gb1;
};

template <typename TO, bool GEN, bool FULL = false>
__global__ __launch_bounds__(512, 2) void k_square_tile4_bf16x3(TileArgs a) {
  __shared__ __align__(16) uint16_t S0[8][2][HPLANE];  // k half 0 of the current K
  __shared__ __align__(16) uint16_t S1[8][2][HPLANE];  // k half 1
  const int64_t t = xcd_tile(a);
  if (t < 0) return;
  const int nbr = a.nbr, W = a.W;
  const int I0 = 4 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t]);
  const int J0 = 4 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t + 1]);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ia = wave >> 1, jp = 2 * (wave & 1);
  const int I = I0 + ia, Jb0 = J0 + jp, Jb1 = J0 + jp + 1;
  int32_t pos0 = -1, pos1 = -1;
  if (I < nbr && Jb0 < nbr && (FULL || I <= Jb0))
    pos0 = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + Jb0]);
  if (I < nbr && Jb1 < nbr && (FULL || I <= Jb1))
    pos1 = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + Jb1]);
  const u32x4 *xq = static_cast<const u32x4 *>(a.xpack);
  const u32x4 *yq = static_cast<const u32x4 *>(GEN ? a.ypack : a.xpack);

  f4 acc0[4][4], acc1[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      acc0[m][n] = f4{0, 0, 0, 0};
      acc1[m][n] = f4{0, 0, 0, 0};
    }

  // K over the union of the 16 blocks' K sets (second pass: operands
  // swapped); the right operand's slots are read along row J of the symmetric
  // slot map.  scan() finds the next non-empty bitmap word (its loads are
  // waited for at once; once per 32 K on dense patterns) and keeps returning
  // false when the K sets are exhausted; issue_k() takes the next K of the
  // word and only issues the loads of its slots, which fin_k() makes
  // wave-uniform after the MFMAs of a k half, so their latency is hidden.
  const uint32_t *lbits = a.bits, *rbits = GEN ? a.ybits : a.bits;
  int wi = -1, pass = 0;
  uint32_t mask = 0u;
  auto scan = [&]() -> bool {
    while (mask == 0u) {
      ++wi;
      if (wi >= W) {
        if (!GEN || pass + 1 >= a.npass) {
          wi = W;
          return false;
        }
        ++pass;
        wi = -1;
        lbits = a.ybits;
        rbits = a.bits;
        continue;
      }
      uint32_t ra = 0u, rb = 0u;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (I0 + r < nbr) ra |= lbits[(int64_t)(I0 + r) * W + wi];
        if (J0 + r < nbr) rb |= rbits[(int64_t)(J0 + r) * W + wi];
      }
      mask = (uint32_t)__builtin_amdgcn_readfirstlane((int)(ra & rb));
    }
    return true;
  };
  // a zero the compiler takes for a per-lane value: the slot loads then stay
  // vector loads into registers, unwaited until fin_k
  int vz = 0;
  asm volatile("" : "+v"(vz));
  const int Rd = wave < 4 ? I0 + wave : J0 + wave - 4;  // the operand this wave loads
  auto issue_k = [&](Stage4 &q) {  // requires mask != 0
    const int K = wi * 32 + __builtin_ctz(mask);
    mask &= mask - 1u;
    q.K = K;
    q.kp = pass;
    const int32_t *li = ((GEN && pass) ? a.yidxmap : a.idxmap) + vz;
    const int32_t *ri = (GEN ? (pass ? a.idxmap : a.yidxmap) : a.idxmap) + vz;
    const bool la = GEN && (pass ? a.yanti : a.xanti), rn = GEN && (pass ? a.xanti : a.yanti);
    const bool ng = GEN && pass && a.neg2;
    constexpr uint32_t SGN2 = 0x80008000u;
    q.sa = li[(int64_t)(I < nbr ? I : 0) * nbr + K];
    q.sb0 = ri[(int64_t)(Jb0 < nbr ? Jb0 : 0) * nbr + K];
    q.sb1 = ri[(int64_t)(Jb1 < nbr ? Jb1 : 0) * nbr + K];
    q.sd = (wave < 4 ? li : ri)[(int64_t)(Rd < nbr ? Rd : 0) * nbr + K];
    q.ga = ((la && I > K) != ng) ? SGN2 : 0u;
    q.gb0 = (rn && K > Jb0) ? SGN2 : 0u;
    q.gb1 = (rn && K > Jb1) ? SGN2 : 0u;
  };
  auto fin_k = [&](Stage4 &q) {  // rows past the last block row read row 0: -1
    q.sa = I < nbr ? __builtin_amdgcn_readfirstlane(q.sa) : -1;
    q.sb0 = Jb0 < nbr ? __builtin_amdgcn_readfirstlane(q.sb0) : -1;
    q.sb1 = Jb1 < nbr ? __builtin_amdgcn_readfirstlane(q.sb1) : -1;
    q.sd = Rd < nbr ? __builtin_amdgcn_readfirstlane(q.sd) : -1;
  };

  // k half kh of the 8 operand images of q into stage st: 64 load
  // instructions of 1 KB (operand o, plane pl, 16-row group rg); wave w issues
  // the 8 of operand w.  Lane l fills row 16 rg + l / 4, chunk l % 4 of the
  // group with the global chunk of logical k chunk (l % 4) ^ swz(row) (swz
  // depends on row % 16 only).
  const uint32_t loff = (uint32_t)(((lane >> 2) * 8 + ((lane & 3) ^ swz(lane >> 2))) * 16);
  auto dma = [&](const Stage4 &q, int kh, uint16_t (*st)[2][HPLANE]) {
    const u32x4 *base = ((wave < 4) == !(GEN && q.kp)) ? xq : yq;
    const int32_t so = q.sd > 0 ? q.sd : 0;  // absent: slot 0, never multiplied
    const bool nimg = wave < 4 ? (FULL || I0 + wave <= q.K) : (!FULL && q.K > J0 + wave - 4);
    const char *img =
        reinterpret_cast<const char *>(base + (int64_t)so * BLK_Q + (nimg ? 0 : IMG_Q) + kh * 4);
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
      for (int rg = 0; rg < 4; ++rg)
        __builtin_amdgcn_global_load_lds(img + pl * 8192 + rg * 2048 + loff, &st[wave][pl][rg * 16 * 32], 16, 0,
                                         0);
  };

  // one k half: per output block the 16 accumulator tiles take lo*hi, then
  // hi*hi, then hi*lo.  Six fragment groups (A lo, B0 hi, B1 hi, A hi, B1 lo,
  // B0 lo) in two A and two B register sets; each group is read from LDS one
  // 16-MFMA step before its first use, so the reads run under the MFMAs.
  const int l16 = lane & 15, g = lane >> 4;
  const int foff = l16 * 32 + ((g ^ swz(l16)) << 3);  // fragment of tile t at foff + 512 t
  int nk0 = 0, nk1 = 0;
  auto compute = [&](const Stage4 &q, uint16_t (*st)[2][HPLANE]) {
    const bool act0 = pos0 >= 0 && q.sa >= 0 && q.sb0 >= 0;
    const bool act1 = pos1 >= 0 && q.sa >= 0 && q.sb1 >= 0;
    nk0 += act0 ? 1 : 0;
    nk1 += act1 ? 1 : 0;
    if (!act0 && !act1) return;
    const uint16_t *ah = st[ia][0], *al = st[ia][1];
    const uint16_t *b0h = st[4 + jp][0], *b0l = st[4 + jp][1], *b1h = st[5 + jp][0], *b1l = st[5 + jp][1];
    u32x4 fa0[4], fa1[4], fb0[4], fb1[4];
    auto ld = [&](u32x4(&f)[4], const uint16_t *pl, uint32_t sg) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f[t] = *reinterpret_cast<const u32x4 *>(pl + foff + 512 * t);
        if (GEN) f[t] ^= u32x4{sg, sg, sg, sg};
      }
    };
    auto mm = [&](f4(&ac)[4][4], const u32x4(&fa)[4], const u32x4(&fb)[4]) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) ac[m][n] = mfma_bf16(fa[m], fb[n], ac[m][n]);
    };
    ld(fa0, al, q.ga);
    if (act0) ld(fb0, b0h, q.gb0);
    if (act1) ld(fb1, b1h, q.gb1);
    if (act0) mm(acc0, fa0, fb0);  // block 0: lo*hi
    ld(fa1, ah, q.ga);
    if (act1) mm(acc1, fa0, fb1);  // block 1: lo*hi
    if (act1) {
      mm(acc1, fa1, fb1);  // block 1: hi*hi
      ld(fb1, b1l, q.gb1);
    }
    if (act0) {
      mm(acc0, fa1, fb0);  // block 0: hi*hi
      ld(fb0, b0l, q.gb0);
    }
    if (act1) mm(acc1, fa1, fb1);  // block 1: hi*lo
    if (act0) mm(acc0, fa1, fb0);  // block 0: hi*lo
  };

  Stage4 q, qn;
  if (scan()) {
    issue_k(q);
    fin_k(q);
    dma(q, 0, S0);
    while (true) {
      __syncthreads();  // k half 0 of K in S0 (every wave waited for its loads); S1 free
      dma(q, 1, S1);
      // the next K of the current bitmap word: its slot loads run under the MFMAs
      bool more = mask != 0u;
      if (more) issue_k(qn);
      compute(q, S0);
      if (more) {
        fin_k(qn);
      } else if (scan()) {  // a new bitmap word (its loads waited for here)
        more = true;
        issue_k(qn);
        fin_k(qn);
      }
      __syncthreads();  // k half 1 in S1; S0 free
      if (more) dma(qn, 0, S0);
      compute(q, S1);
      if (!more) break;
      q = qn;
    }
  }
  // f32 16 x 16 accumulator layout: element v of lane group g is row 4 g + v;
  // nk counted both k halves of every K
  const auto rowf = [](int gg, int qq) { return 4 * gg + qq; };
  // Block 1's accumulators wait in the (now idle) LDS stages, 16 KB per wave,
  // while block 0's epilogue runs, so the two never hold registers at once
  // (8 waves leave 256 registers per lane; both blocks plus the FP64
  // epilogue do not fit).
  __syncthreads();  // every wave is done with S0 / S1
  f4 *park = reinterpret_cast<f4 *>(wave < 4 ? &S0[0][0][0] : &S1[0][0][0]) + (wave & 3) * 1024;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) park[(m * 4 + n) * 64 + lane] = acc1[m][n];
  if (pos0 >= 0) square_epilogue<float, TO>(acc0, a, I, Jb0, pos0, nk0 / 2, rowf);
  asm volatile("" ::: "memory");  // keep the reload below block 0's epilogue
  f4 acc2[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc2[m][n] = park[(m * 4 + n) * 64 + lane];
  if (pos1 >= 0) square_epilogue<float, TO>(acc2, a, I, Jb1, pos1, nk1 / 2, rowf);
}

}  // namespace

void launch_pack_bf16x3(Ctx &c, const float *pool, const int32_t *slot, int64_t nblocks, uint16_t *packed) {
  if (nblocks <= 0) return;
  k_pack_bf16x3<<<(unsigned)nblocks, TPB, 0, c.stream>>>(pool, slot, nblocks, packed);
  SP2_LAUNCH_CHECK();
}

void launch_square_tile_bf16x3(Ctx &c, const TileArgs &a) {
  if (a.ntiles <= 0) return;
  if (a.xprec != P32) fail(SP2_ERR_INVALID_ARG, "BF16x3 square needs an FP32 input pool");
  const bool gen = a.ypool != a.xpool || a.npass != 1 || a.xanti || a.yanti;
  if (!a.xpack || (gen && !a.ypack)) fail(SP2_ERR_INVALID_ARG, "BF16x3 square needs packed operands");
  const unsigned g = (unsigned)(8 * a.xcd_chunk);
  if (a.full) {
    if (!a.ypack || a.npass != 1 || a.xanti || a.yanti || a.oprec != P32)
      fail(SP2_ERR_INVALID_ARG, "general-storage BF16x3 product: one pass, FP32 output, both operands");
    if (a.tb == 4)
      k_square_tile4_bf16x3<float, true, true><<<g, 512, 0, c.stream>>>(a);
    else
      k_square_tile_bf16x3<float, true, true><<<g, TPB, 0, c.stream>>>(a);
    SP2_LAUNCH_CHECK();
    return;
  }
  if (a.tb == 4) {
    if (a.oprec == P32) {
      if (gen)
        k_square_tile4_bf16x3<float, true><<<g, 512, 0, c.stream>>>(a);
      else
        k_square_tile4_bf16x3<float, false><<<g, 512, 0, c.stream>>>(a);
    } else {
      if (gen)
        k_square_tile4_bf16x3<double, true><<<g, 512, 0, c.stream>>>(a);
      else
        k_square_tile4_bf16x3<double, false><<<g, 512, 0, c.stream>>>(a);
    }
    SP2_LAUNCH_CHECK();
    return;
  }
  if (a.tb != 2) fail(SP2_ERR_INVALID_ARG, "BF16x3 square: tile edge must be 2 or 4 blocks");
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
