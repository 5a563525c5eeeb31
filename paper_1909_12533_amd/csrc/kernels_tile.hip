// Tiled numeric block-sparse symmetric square (the hot kernel of Algorithm 2)
// with the polynomial update, idempotency error and traces in its epilogue.
//
// Work decomposition: one workgroup per 2 x 2 tile of output blocks
// (I0, I0+1) x (J0, J0+1), I0 <= J0 in tile units; wave w computes the whole
// 64 x 64 output block (I0 + w / 2, J0 + w % 2) as 4 x 4 MFMA 16 x 16 tiles.
// The K loop runs over the set bits of (bits[I0] | bits[I0+1]) &
// (bits[J0] | bits[J0+1]), which is exactly the union of the four blocks'
// K sets.  Per K the four operand blocks X_{I0,K}, X_{I0+1,K}, X_{K,J0},
// X_{K,J0+1} are staged through LDS once and each is used by two waves, so
// every 32 KB loaded from global memory feeds 2 x 64^3 x 2 flops; a wave
// whose own pair of blocks is absent for this K skips its MFMAs.  Lower
// blocks X_KI (K > I) are read as transposes of the stored X_IK by the
// fragment addressing.  The next K's four blocks are loaded into registers
// while the current K's MFMAs run.
#include "mfma.h"

namespace sp2 {

namespace {

using namespace dev;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-deep k chunk fragments for a wave computing MT 16-row tiles (rows
// r0 + 16 m) of a 64 x 64 block and all four 16-column tiles: k index
// k0 + 4 g + s for MFMA s of the chunk (lane group g = lane / 16).
template <typename T, bool TA, bool TB, int MT> struct Frag {
  T a[MT][4], b[4][4];
  __device__ inline void load(const T *As, const T *Bs, int k0, int r0) {
    constexpr int LD = MF<T>::LD;
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15, kb = k0 + 4 * (lane >> 4);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int r = r0 + 16 * m + l16;
      if (!TA) {
        const T *p = As + r * LD + kb;
#pragma unroll
        for (int s = 0; s < 4; ++s) a[m][s] = p[s];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[m][s] = As[(kb + s) * LD + r];
      }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int c = 16 * n + l16;
      if (TB) {
        const T *p = Bs + c * LD + kb;
#pragma unroll
        for (int s = 0; s < 4; ++s) b[n][s] = p[s];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) b[n][s] = Bs[(kb + s) * LD + c];
      }
    }
  }
};

template <typename T, bool TA, bool TB, int MT>
__device__ inline void mma_full(typename MF<T>::acc_t (&acc)[MT][4], const T *As, const T *Bs, int r0) {
  Frag<T, TA, TB, MT> f;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    f.load(As, Bs, 16 * kc, r0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = MF<T>::op(f.a[m][s], f.b[n][s], acc[m][n]);
  }
}

template <typename T, int MT>
__device__ inline void mma_dispatch(typename MF<T>::acc_t (&acc)[MT][4], const T *As, const T *Bs, bool tA, bool tB,
                                    int r0) {
  if (!tA && !tB)
    mma_full<T, false, false, MT>(acc, As, Bs, r0);
  else if (!tA && tB)
    mma_full<T, false, true, MT>(acc, As, Bs, r0);
  else if (tA && !tB)
    mma_full<T, true, false, MT>(acc, As, Bs, r0);
  else
    mma_full<T, true, true, MT>(acc, As, Bs, r0);
}

// GEN: general product (second operand Y, optional second pass with the
// roles swapped, sign flips of antisymmetric lower blocks); otherwise the
// square X X with the same code minus that bookkeeping.
// NW = 4: one wave per output block (all 4 x 4 MFMA tiles); NW = 8: two waves
// per output block, each with the 2 x 4 tiles of rows 32 h .. 32 h + 31, so
// that every SIMD holds two waves (one multiplies while the other waits on LDS).
// TI: element type of the stored operands (and of G); T = double with
// TI = float multiplies FP32-stored values in FP64 (each value widened
// exactly when it is written to LDS).
template <typename T, typename TO, bool GEN, int NW, typename TI = T>
__global__ __launch_bounds__(64 * NW, (NW == 4 && sizeof(T) == 4) ? 2 : 1) void k_square_tile(TileArgs a) {
  static_assert(sizeof(TI) <= sizeof(T), "operands are widened, never narrowed");
  constexpr int LD = MF<T>::LD;
  constexpr int NT = 64 * NW;      // threads
  constexpr int MT = 16 / NW;      // 16-row A tiles per wave
  __shared__ __align__(16) T As[2][64 * LD];
  __shared__ __align__(16) T Bs[2][64 * LD];
  __shared__ double red[4][4];     // NW = 8: partial sums of the second-half waves
  const int64_t t = xcd_tile(a);
  if (t < 0) return;
  const int nbr = a.nbr, W = a.W;
  const int I0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t]);
  const int J0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t + 1]);
  const int wave = threadIdx.x >> 6;
  const int blk = wave & 3, half = wave >> 2;
  const int row0 = NW == 8 ? 32 * half : 0;
  const int ia = blk >> 1, jb = blk & 1;
  const int I = I0 + ia, J = J0 + jb;
  const bool has_i1 = I0 + 1 < nbr, has_j1 = J0 + 1 < nbr;
  int32_t pos = -1;
  if (I < nbr && J < nbr && I <= J) pos = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + J]);

  typename MF<T>::acc_t acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = typename MF<T>::acc_t{0, 0, 0, 0};

  // K over the union of the four blocks' K sets (rows I0, I0+1 of the left
  // operand, columns J0, J0+1 of the right one); with two passes the scan
  // restarts with the operands swapped
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

  // staged operand blocks A0 = L_{I0,K}, A1 = L_{I0+1,K}, B0 = R_{K,J0}, B1 = R_{K,J0+1}
  // with (L, R) = (X, Y) in the first pass and (Y, X) in the second
  constexpr int EPC = Stage<TI>::EPC;            // stored elements per 16-byte chunk
  constexpr int NCH = BB / EPC / NT;             // 16-byte chunks per thread and block
  constexpr int QB = BB * (int)sizeof(TI) / 16;  // 16-byte chunks per block
  constexpr uint32_t SGN = 0x80000000u;
  const u32x4 *xq = reinterpret_cast<const u32x4 *>(a.xpool);
  const u32x4 *yq = reinterpret_cast<const u32x4 *>(GEN ? a.ypool : a.xpool);
  u32x4 r0[NCH], r1[NCH], r2[NCH], r3[NCH];
  int32_t s0 = -1, s1 = -1, s2 = -1, s3 = -1;
  uint32_t g0 = 0u, g1 = 0u, g2 = 0u, g3 = 0u;  // sign bit to flip per staged block
// absent block (slot < 0): zeros, and no load is issued (wave-uniform branch)
#define SP2_LOAD_BLOCK(R, Q, SL)                                                  \
  do {                                                                            \
    if ((SL) >= 0) {                                                              \
      const u32x4 *src_ = (Q) + (int64_t)(SL) * QB + threadIdx.x;                 \
      _Pragma("unroll") for (int j = 0; j < NCH; ++j) R[j] = src_[j * NT];        \
    } else {                                                                      \
      _Pragma("unroll") for (int j = 0; j < NCH; ++j) R[j] = u32x4{0u, 0u, 0u, 0u}; \
    }                                                                             \
  } while (0)
#define SP2_ISSUE(KK, KP)                                                                                  \
  do {                                                                                                     \
    const int32_t *li_ = (GEN && (KP)) ? a.yidxmap : a.idxmap;                                             \
    const int32_t *ri_ = GEN ? ((KP) ? a.idxmap : a.yidxmap) : a.idxmap;                                   \
    const u32x4 *lq_ = (GEN && (KP)) ? yq : xq, *rq_ = (GEN && (KP)) ? xq : yq;                            \
    s0 = __builtin_amdgcn_readfirstlane(li_[(int64_t)I0 * nbr + (KK)]);                                    \
    s1 = has_i1 ? __builtin_amdgcn_readfirstlane(li_[(int64_t)(I0 + 1) * nbr + (KK)]) : -1;                \
    s2 = __builtin_amdgcn_readfirstlane(ri_[(int64_t)(KK) * nbr + J0]);                                    \
    s3 = has_j1 ? __builtin_amdgcn_readfirstlane(ri_[(int64_t)(KK) * nbr + J0 + 1]) : -1;                  \
    if (GEN) {                                                                                             \
      const bool la_ = (KP) ? a.yanti : a.xanti, ra_ = (KP) ? a.xanti : a.yanti;                           \
      const bool ng_ = (KP) && a.neg2;                                                                     \
      g0 = ((la_ && I0 > (KK)) != ng_) ? SGN : 0u;                                                         \
      g1 = ((la_ && I0 + 1 > (KK)) != ng_) ? SGN : 0u;                                                     \
      g2 = (ra_ && (KK) > J0) ? SGN : 0u;                                                                  \
      g3 = (ra_ && (KK) > J0 + 1) ? SGN : 0u;                                                              \
    }                                                                                                      \
    SP2_LOAD_BLOCK(r0, lq_, s0);                                                                           \
    SP2_LOAD_BLOCK(r1, lq_, s1);                                                                           \
    SP2_LOAD_BLOCK(r2, rq_, s2);                                                                           \
    SP2_LOAD_BLOCK(r3, rq_, s3);                                                                           \
  } while (0)

  int nk = 0;
  int K = next_k();
  if (K >= 0) SP2_ISSUE(K, kpass);
  while (K >= 0) {
    const int32_t c0 = s0, c1 = s1, c2 = s2, c3 = s3;
    __syncthreads();  // previous tiles fully consumed
    if constexpr (sizeof(TI) < sizeof(T)) {
      // FP32-stored values, FP64 arithmetic: 4 floats per chunk, widened
      // (exactly) to 4 doubles, sign flips applied to the floats first
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int e = (j * NT + (int)threadIdx.x) * EPC;
        const int o = (e >> 6) * LD + (e & 63);
        const u32x4 w[4] = {r0[j] ^ u32x4{g0, g0, g0, g0}, r1[j] ^ u32x4{g1, g1, g1, g1},
                            r2[j] ^ u32x4{g2, g2, g2, g2}, r3[j] ^ u32x4{g3, g3, g3, g3}};
        T *dst[4] = {&As[0][o], &As[1][o], &Bs[0][o], &Bs[1][o]};
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) dst[b][v] = (T)__uint_as_float(w[b][v]);
      }
    } else if (GEN) {
      // sign flips on the staged words (FP64: the high word of each double)
      const uint32_t lo0 = sizeof(T) == 8 ? 0u : g0, lo1 = sizeof(T) == 8 ? 0u : g1;
      const uint32_t lo2 = sizeof(T) == 8 ? 0u : g2, lo3 = sizeof(T) == 8 ? 0u : g3;
      const u32x4 m0 = u32x4{lo0, g0, lo0, g0}, m1 = u32x4{lo1, g1, lo1, g1};
      const u32x4 m2 = u32x4{lo2, g2, lo2, g2}, m3 = u32x4{lo3, g3, lo3, g3};
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int e = (j * NT + (int)threadIdx.x) * EPC;
        const int o = (e >> 6) * LD + (e & 63);
        *reinterpret_cast<u32x4 *>(&As[0][o]) = r0[j] ^ m0;
        *reinterpret_cast<u32x4 *>(&As[1][o]) = r1[j] ^ m1;
        *reinterpret_cast<u32x4 *>(&Bs[0][o]) = r2[j] ^ m2;
        *reinterpret_cast<u32x4 *>(&Bs[1][o]) = r3[j] ^ m3;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int e = (j * NT + (int)threadIdx.x) * EPC;
        const int o = (e >> 6) * LD + (e & 63);
        *reinterpret_cast<u32x4 *>(&As[0][o]) = r0[j];
        *reinterpret_cast<u32x4 *>(&As[1][o]) = r1[j];
        *reinterpret_cast<u32x4 *>(&Bs[0][o]) = r2[j];
        *reinterpret_cast<u32x4 *>(&Bs[1][o]) = r3[j];
      }
    }
    __syncthreads();
    const int Kn = next_k();
    if (Kn >= 0) SP2_ISSUE(Kn, kpass);  // next K's blocks in flight during the MFMAs
    const int32_t sa = ia ? c1 : c0, sb = jb ? c3 : c2;
    if (pos >= 0 && sa >= 0 && sb >= 0) {
      mma_dispatch<T, MT>(acc, ia ? As[1] : As[0], jb ? Bs[1] : Bs[0], I > K, K > J, row0);
      ++nk;
    }
    K = Kn;
  }
#undef SP2_ISSUE
#undef SP2_LOAD_BLOCK
  const auto rowf = [](int g, int q) { return MF<T>::row(g, q); };
  if constexpr (NW == 4) {
    if (pos < 0) return;
    square_epilogue<TI, TO>(acc, a, I, J, pos, nk, rowf);
  } else {
  // two waves per block: the second half's partial sums are added (in a fixed
  // order) by the first half's wave
  EpiSums ps{};
  if (pos >= 0) ps = epilogue_rows<TI, TO, MT>(acc, a, I, J, pos, row0, rowf);
  const int lane = threadIdx.x & 63;
  if (half == 1 && lane == 0) {
    red[blk][0] = ps.e2;
    red[blk][1] = ps.tx;
    red[blk][2] = ps.ts;
    red[blk][3] = ps.nr;
  }
  __syncthreads();
  if (half == 0 && lane == 0 && pos >= 0) {
    double *p = a.parts + (int64_t)pos * NPART;
    p[0] = ps.e2 + red[blk][0];
    p[1] = ps.tx + red[blk][1];
    p[2] = ps.ts + red[blk][2];
    p[3] = ps.nr + red[blk][3];
    p[4] = (double)nk;
  }
  }
}

// Tile order: super-tiles of ST x ST tiles (2 ST x 2 ST output blocks) in
// row-major order, tiles row-major inside a super-tile.  Linear id
// ((STI * nst + STJ) * ST + ti) * ST + tj with TI = STI * ST + ti,
// TJ = STJ * ST + tj.
#ifndef SP2_TILE_ST
#define SP2_TILE_ST 4
#endif
constexpr int ST = SP2_TILE_ST;

__device__ inline bool tile_of(int64_t id, int ntr, int nst, bool full, int &TI, int &TJ) {
  const int tj = (int)(id % ST);
  const int64_t r1 = id / ST;
  const int ti = (int)(r1 % ST);
  const int64_t r2 = r1 / ST;
  const int STJ = (int)(r2 % nst), STI = (int)(r2 / nst);
  TI = STI * ST + ti;
  TJ = STJ * ST + tj;
  return TI < ntr && TJ < ntr && (full || TI <= TJ);
}

// flags of tb x tb output tiles holding at least one output block
__global__ void k_tile_flags(const int32_t *oidx, int nbr, int tb, int ntr, int nst, int64_t nid, bool full,
                             int64_t *flag) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= nid) return;
  int TI, TJ;
  int64_t f = 0;
  if (tile_of(id, ntr, nst, full, TI, TJ)) {
    for (int a = 0; a < tb; ++a)
      for (int b = 0; b < tb; ++b) {
        const int I = tb * TI + a, J = tb * TJ + b;
        if (I < nbr && J < nbr && (full || I <= J) && oidx[(int64_t)I * nbr + J] >= 0) f = 1;
      }
  }
  flag[id] = f;
}

__global__ void k_tile_write(const int64_t *flag, const int64_t *pos, int ntr, int nst, int64_t nid, bool full,
                             int32_t *tiles) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= nid || !flag[id]) return;
  int TI, TJ;
  tile_of(id, ntr, nst, full, TI, TJ);
  const int64_t o = pos[id];
  tiles[2 * o] = TI;
  tiles[2 * o + 1] = TJ;
}

}  // namespace

int64_t build_tiles(Ctx &c, const int32_t *oidx, int nbr, Buf &tiles, int tb, bool full) {
  if (tb != 2 && tb != 4) fail(SP2_ERR_INVALID_ARG, "tile edge must be 2 or 4 blocks");
  const int ntr = (nbr + tb - 1) / tb;
  const int nst = (ntr + ST - 1) / ST;
  const int64_t nid = (int64_t)nst * nst * ST * ST;
  Buf flag = c.alloc(sizeof(int64_t) * nid), pos = c.alloc(sizeof(int64_t) * (nid + 1));
  k_tile_flags<<<(unsigned)((nid + TPB - 1) / TPB), TPB, 0, c.stream>>>(oidx, nbr, tb, ntr, nst, nid, full,
                                                                        flag.as<int64_t>());
  SP2_LAUNCH_CHECK();
  scan_exclusive_i64(c, flag.as<int64_t>(), pos.as<int64_t>(), nid);
  int64_t nt = 0;
  c.d2h(&nt, pos.as<int64_t>() + nid, sizeof(int64_t));
  tiles = c.alloc(sizeof(int32_t) * 2 * (nt > 0 ? nt : 1));
  k_tile_write<<<(unsigned)((nid + TPB - 1) / TPB), TPB, 0, c.stream>>>(flag.as<int64_t>(), pos.as<int64_t>(), ntr, nst,
                                                                        nid, full, tiles.as<int32_t>());
  SP2_LAUNCH_CHECK();
  return nt;
}

void launch_square_tile(Ctx &c, int mode, const TileArgs &a) {
  if (a.ntiles <= 0) return;
  if (a.full) fail(SP2_ERR_INVALID_ARG, "register-staged tiled kernel: symmetric storage only");
  if (a.tb != 2 && mode != M_BF16X3) fail(SP2_ERR_INVALID_ARG, "4 x 4 tiles are for the BF16x3 square only");
  const bool gen = a.ypool != a.xpool || a.npass != 1 || a.xanti || a.yanti;
  if (gen && !(a.ypool && a.yidxmap && a.ybits && (a.npass == 1 || a.npass == 2)))
    fail(SP2_ERR_INVALID_ARG, "tiled product: incomplete second operand");
  const unsigned g = (unsigned)(8 * a.xcd_chunk);
  if (mode == M_F64 && a.xprec == P32) {
    // FP64 arithmetic on FP32-stored values, FP32 result (the FP64 tail of an
    // expansion whose FP64 iterates do not fit in device memory)
    if (gen || a.oprec != P32) fail(SP2_ERR_INVALID_ARG, "FP64 square of FP32 values: square only, FP32 result");
    k_square_tile<double, float, false, 8, float><<<g, 512, 0, c.stream>>>(a);
  } else if (mode == M_F64) {
    if (a.oprec == P32) {  // FP64 arithmetic, result rounded to FP32 (the correction's commutator)
      if (!gen) fail(SP2_ERR_INVALID_ARG, "FP64 square with FP32 output is for products only");
      k_square_tile<double, float, true, 8><<<g, 512, 0, c.stream>>>(a);
    } else if (gen) {
      k_square_tile<double, double, true, 8><<<g, 512, 0, c.stream>>>(a);
    } else {
      k_square_tile<double, double, false, 8><<<g, 512, 0, c.stream>>>(a);
    }
  } else if (mode == M_F32) {
    if (a.xprec != P32) fail(SP2_ERR_INVALID_ARG, "FP32 square needs an FP32 input pool");
    if (a.oprec == P32) {
      if (gen)
        k_square_tile<float, float, true, 4><<<g, TPB, 0, c.stream>>>(a);
      else
        k_square_tile<float, float, false, 4><<<g, TPB, 0, c.stream>>>(a);
    } else {
      if (gen)
        k_square_tile<float, double, true, 4><<<g, TPB, 0, c.stream>>>(a);
      else
        k_square_tile<float, double, false, 4><<<g, TPB, 0, c.stream>>>(a);
    }
  } else if (mode == M_BF16X3) {
    launch_square_tile_bf16x3(c, a);
    return;
  } else {
    fail(SP2_ERR_INVALID_ARG, "unknown square mode");
  }
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
