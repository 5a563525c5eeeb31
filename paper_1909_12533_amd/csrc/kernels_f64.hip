// FP64 squares and two-operand products with operands loaded straight to LDS
// (the symmetric square of Algorithm 2 in the method's reference arithmetic;
// the products X Y +- Y X of the adjoint and the correction; the FP64 square
// of FP32-stored iterates, widened to FP64 at the fragment reads).
//
// One workgroup of four waves per 2 x 2 tile of output blocks; wave w owns the
// whole 64 x 64 block (I0 + w / 2, J0 + w % 2) in 4 x 4 MFMA accumulator tiles.
// K runs ascending over the union of the tile's K sets and each K is taken in
// four 16-deep k quarters, so every output element accumulates in the same
// order as in k_square_tile<double, TO, GEN, 8> (K ascending, the second
// pass after the first, 16-deep k chunks in order, k = 4 g + s within an
// MFMA): the two give bit-identical results, the block sums included (added
// over rows 0..31 and 32..63 in that order).  Sign flips of antisymmetric
// lower blocks and of a subtracted second pass are exact negations of the
// fragments after their LDS read.
//
// Staging: each quarter of the four operand blocks (A0, A1, B0, B1; 8 KB
// each) is loaded by global_load_lds_dwordx4 straight into LDS, wave w
// loading operand w; quarters alternate between two stages (64 KB in all, so
// two workgroups share a CU and one computes while the other waits at a
// barrier), and the load of the next quarter runs under the MFMAs of the
// current one.  The slot lookups of the next K are issued before the MFMAs of
// a quarter and consumed after them.
//
// A staged quarter of a stored 64 x 64 block is either its 16 columns k, as
// [64 rows][16 k] (128-byte rows, "kcol": the operand is used untransposed
// along k) or its 16 rows k, as [16 k][64 columns] (512-byte rows, "krow":
// used transposed).  The 16-byte chunks of each row are XOR-swizzled so that
// the fragment reads of 16 lanes hit distinct banks:
//   kcol: chunk c of row r at position c ^ ((r >> 1) & 7);
//   krow: chunk c of k-row kr at position c ^ (8 * ((kr >> 2) & 1)).
// One load instruction writes 1 KB of LDS contiguously (lane l at byte 16 l):
// 8 kcol rows or 2 krow rows; each lane fetches the global chunk that belongs
// at its position.
#include "mfma.h"

namespace sp2 {

namespace {

using namespace dev;


// Staging geometry of a quarter slice (16 k) of one 64 x 64 operand block
// stored as TI: kcol [64 rows][16 k] (the operand used untransposed along k),
// krow [16 k][64 columns] (used transposed), 16-byte chunks XOR-swizzled so
// that the fragment reads of the 16 lanes of a lane group hit distinct banks.
// One load instruction writes 1 KB of LDS contiguously (lane l at byte 16 l);
// each lane fetches the global chunk that belongs at its position.
template <typename TI> struct QGeom;
template <> struct QGeom<double> {
  static constexpr int BYTES = 64 * 16 * 8;  // 8 KB per operand quarter
  static constexpr int LOADS = BYTES / 1024;
  static constexpr int PAIR_KCOL = 8, PAIR_KROW = 512;  // byte distance of elements k and k + 1
  // kcol: 128-byte rows, chunk c of row r at c ^ ((r >> 1) & 7); krow:
  // 512-byte rows, chunk c of k-row kr at c ^ (8 ((kr >> 2) & 1))
  __device__ static int col_pos(int r, int c) { return c ^ ((r >> 1) & 7); }
  __device__ static int row_pos(int kr, int c) { return c ^ (((kr >> 2) & 1) << 3); }
  // byte offset of element (r, k), k even
  __device__ static int frag(bool kcol, int r, int k) {
    return kcol ? 16 * (r * 8 + col_pos(r, k >> 1)) : 8 * (k * 64 + row_pos(k, r >> 1) * 2 + (r & 1));
  }
  // global 16-byte chunk (within the block) that load i of lane l brings to quarter kq
  __device__ static int gchunk(bool kcol, int kq, int i, int lane) {
    if (kcol) {
      const int r = 8 * i + (lane >> 3), p = lane & 7;
      return r * 32 + 8 * kq + col_pos(r, p);
    }
    const int kr = 2 * i + (lane >> 5), p = lane & 31;
    return (16 * kq + kr) * 32 + row_pos(kr, p);
  }
};
template <> struct QGeom<float> {
  static constexpr int BYTES = 64 * 16 * 4;  // 4 KB per operand quarter
  static constexpr int LOADS = BYTES / 1024;
  static constexpr int PAIR_KCOL = 4, PAIR_KROW = 256;
  // kcol: 64-byte rows, chunk c (4 k) of row r at c ^ ((r >> 2) & 3); krow:
  // 256-byte rows, chunk c (4 columns) of k-row kr at c ^ (4 ((kr >> 2) & 3))
  __device__ static int col_pos(int r, int c) { return c ^ ((r >> 2) & 3); }
  __device__ static int row_pos(int kr, int c) { return c ^ (((kr >> 2) & 3) << 2); }
  __device__ static int frag(bool kcol, int r, int k) {
    return kcol ? 16 * (r * 4 + col_pos(r, k >> 2)) + 4 * (k & 3) : 16 * (k * 16 + row_pos(k, r >> 2)) + 4 * (r & 3);
  }
  __device__ static int gchunk(bool kcol, int kq, int i, int lane) {
    if (kcol) {
      const int r = 16 * i + (lane >> 2), p = lane & 3;
      return r * 16 + 4 * kq + col_pos(r, p);
    }
    const int kr = 4 * i + (lane >> 4), p = lane & 15;
    return (16 * kq + kr) * 16 + row_pos(kr, p);
  }
};

// One quarter of MFMAs for the wave's 64 x 64 block: 4 x 4 accumulator tiles,
// k = 4 g + s (lane group g = lane / 16, MFMA s = 0..3), fragments read in
// pairs s = 2 sp, 2 sp + 1 and widened from the stored TI to FP64.
// The orientation of each operand is a run-time choice of per-lane offsets
// (one code path: the accumulators stay in place).  Every read is one byte
// offset from the stage array: the compiler tells reads of one stage from the
// loads still landing in the other only for addresses it can trace to the
// array in a few steps.
template <typename TI>
__device__ __forceinline__ void mma_quarter(d4 (&acc)[4][4], const char *st, int oa, int ob, bool ka, bool kb,
                                            bool na, bool nb, int lane) {
  using G = QGeom<TI>;
  const int l16 = lane & 15;
  const int da = ka ? G::PAIR_KCOL : G::PAIR_KROW, db = kb ? G::PAIR_KCOL : G::PAIR_KROW;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    const int k = 4 * (lane >> 4) + 2 * sp;
    double fa[4][2], fb[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int o = oa + G::frag(ka, 16 * m + l16, k);
      fa[m][0] = (double)*reinterpret_cast<const TI *>(st + o);
      fa[m][1] = (double)*reinterpret_cast<const TI *>(st + o + da);
      if (na) {
        fa[m][0] = -fa[m][0];
        fa[m][1] = -fa[m][1];
      }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int o = ob + G::frag(kb, 16 * n + l16, k);
      fb[n][0] = (double)*reinterpret_cast<const TI *>(st + o);
      fb[n][1] = (double)*reinterpret_cast<const TI *>(st + o + db);
      if (nb) {
        fb[n][0] = -fb[n][0];
        fb[n][1] = -fb[n][1];
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = MF<double>::op(fa[m][s], fb[n][s], acc[m][n]);
  }
}

// GEN: general product (second operand Y, a second pass with the roles
// swapped and its sign, antisymmetric operands); otherwise the square X X.
// FULL (with GEN, one pass): general storage, X and Y blocks read as stored
// (X by its direct map, Y by the map of its transpose), output blocks of both
// triangles.
// TI: stored operand values (double, or float: FP32 storage, widened to
// FP64 at the fragment reads); TO: stored result.
template <typename TI, typename TO, bool GEN, bool FULL = false>
__global__ __launch_bounds__(256, 2) void k_square_f64_lds(TileArgs a) {
  using G = QGeom<TI>;
  // even quarters in S0, odd ones in S1: operands A0, A1, B0, B1 at w G::BYTES
  // (arrays sized for FP64 operands whatever TI is: a stage size that depends
  // on the template argument leaves the host-side launch stub undefined)
  __shared__ __align__(16) char S0[4 * QGeom<double>::BYTES];
  __shared__ __align__(16) char S1[4 * QGeom<double>::BYTES];
  const int64_t t = xcd_tile(a);
  if (t < 0) return;
  const int nbr = a.nbr, W = a.W;
  const int I0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t]);
  const int J0 = 2 * __builtin_amdgcn_readfirstlane(a.tiles[2 * t + 1]);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ia = wave >> 1, jb = wave & 1;
  const int I = I0 + ia, J = J0 + jb;
  const bool has_i1 = I0 + 1 < nbr, has_j1 = J0 + 1 < nbr;
  int32_t pos = -1;
  if (I < nbr && J < nbr && (FULL || I <= J)) pos = __builtin_amdgcn_readfirstlane(a.oidx[(int64_t)I * nbr + J]);

  d4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = d4{0, 0, 0, 0};

  // K over the union of the four blocks' K sets (rows I0, I0 + 1 of the left
  // operand, columns J0, J0 + 1 of the right one); with two passes the scan
  // restarts with the operands swapped; once exhausted it keeps returning false
  const uint32_t *ybits = GEN ? a.ybits : a.bits;
  const uint32_t *bI0 = a.bits + (int64_t)I0 * W, *bI1 = a.bits + (int64_t)(has_i1 ? I0 + 1 : I0) * W;
  const uint32_t *bJ0 = ybits + (int64_t)J0 * W, *bJ1 = ybits + (int64_t)(has_j1 ? J0 + 1 : J0) * W;
  int wi = -1, pass = 0;
  uint32_t mask = 0u;
  // staged K as one wave sees it: the slots of its own A and B blocks, the
  // slot of the operand it loads (operand w: A0, A1, B0, B1), the
  // orientations (kcol) of those three, the pass (left operand X, or Y) and
  // the sign flips of the wave's A and B blocks (antisymmetric lower block,
  // subtracted second pass)
  struct StK {
    int K;
    int32_t sa, sb, sd;
    bool ka, kb, kd;
    int kp;
    bool na, nb;
  };
  const int Rd = wave < 2 ? I0 + wave : J0 + wave - 2;  // block row of the operand this wave loads
  // a zero the compiler takes for a per-lane value: the slot loads below then
  // stay in vector registers (and unwaited) until fin_k
  int vz = 0;
  asm volatile("" : "+v"(vz));
  auto next_k = [&](StK &q) -> bool {
    while (mask == 0u) {
      ++wi;
      if (wi >= W) {
        if (!GEN || pass + 1 >= a.npass) {
          wi = W;
          return false;
        }
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
    const int K = wi * 32 + __builtin_ctz(mask);
    mask &= mask - 1u;
    q.K = K;
    // the slot loads are only issued here; fin_k makes them wave-uniform
    // after the MFMAs of a quarter, so their latency is hidden (rows past the
    // last block row read row 0 and are replaced by -1 in fin_k)
    const int kp = GEN ? pass : 0;
    const int32_t *li = (kp ? a.yidxmap : a.idxmap) + vz;
    const int32_t *ri = (GEN ? (kp ? a.idxmap : a.yidxmap) : a.idxmap) + vz;
    q.sa = li[(int64_t)(I < nbr ? I : 0) * nbr + K];
    q.sb = ri[(int64_t)(J < nbr ? J : 0) * nbr + K];
    q.ka = FULL || !(I > K);
    q.kb = !FULL && K > J;
    q.sd = (wave < 2 ? li : ri)[(int64_t)(Rd < nbr ? Rd : 0) * nbr + K];
    q.kd = wave < 2 ? (FULL || !(Rd > K)) : (!FULL && K > Rd);
    q.kp = kp;
    if (GEN && !FULL) {
      const bool la = kp ? a.yanti : a.xanti, ra = kp ? a.xanti : a.yanti;
      q.na = (la && I > K) != (kp && a.neg2);
      q.nb = ra && K > J;
    } else {
      q.na = q.nb = false;
    }
    return true;
  };
  auto fin_k = [&](StK &q) {
    q.sa = I < nbr ? __builtin_amdgcn_readfirstlane(q.sa) : -1;
    q.sb = J < nbr ? __builtin_amdgcn_readfirstlane(q.sb) : -1;
    q.sd = Rd < nbr ? __builtin_amdgcn_readfirstlane(q.sd) : -1;
  };

  // quarter kq (k = 16 kq .. 16 kq + 15) of operand w of q into stage st:
  // G::LOADS load instructions of 1 KB
  const TI *xp = static_cast<const TI *>(a.xpool);
  const TI *yp = static_cast<const TI *>(GEN ? a.ypool : a.xpool);
  auto dma = [&](const StK &q, int kq, char *st) {
    const int32_t so = q.sd >= 0 ? q.sd : 0;  // absent: slot 0, never multiplied
    const TI *pool = ((wave < 2) == !(GEN && q.kp)) ? xp : yp;
    const char *blkp = reinterpret_cast<const char *>(pool + (int64_t)so * BB);
    char *dst = st + wave * G::BYTES;
#pragma unroll
    for (int i = 0; i < G::LOADS; ++i) {
      // the chunk index is taken into a local first: with the template-dependent
      // call inside the builtin's arguments the host pass drops the kernel's stub
      const int gc = G::gchunk(q.kd, kq, i, lane);
      __builtin_amdgcn_global_load_lds(blkp + gc * 16, dst + i * 1024, 16, 0, 0);
    }
  };

  auto compute = [&](const StK &q, const char *st) {
    if (pos < 0 || q.sa < 0 || q.sb < 0) return;
    mma_quarter<TI>(acc, st, ia * G::BYTES, (2 + jb) * G::BYTES, q.ka, q.kb, GEN && q.na, GEN && q.nb, lane);
  };

  // quarters of K alternate between the stages; each iteration of the loop
  // takes quarters 2 h, 2 h + 1 of K and loads the following two
  int nk = 0;
  StK q, qn;
  if (next_k(q)) {
    fin_k(q);
    dma(q, 0, S0);
    int h = 0;
    bool more = true;
    while (true) {
      __syncthreads();  // quarter 2 h in S0 (every wave waited for its loads); S1 free
      if (h == 1) more = next_k(qn);
      dma(q, 2 * h + 1, S1);
      compute(q, S0);
      if (h == 1 && more) fin_k(qn);
      __syncthreads();  // quarter 2 h + 1 in S1; S0 free
      if (h == 0)
        dma(q, 2, S0);
      else if (more)
        dma(qn, 0, S0);
      compute(q, S1);
      if (h == 1) {
        if (pos >= 0 && q.sa >= 0 && q.sb >= 0) ++nk;
        if (!more) break;
        q = qn;
      }
      h ^= 1;
    }
  }
  if (pos < 0) return;
  const auto rowf = [](int g, int v) { return MF<double>::row(g, v); };
  // the block's sums over rows 0..31 and 32..63 separately, added in that
  // order (the same rounding as two waves of 32 rows each)
  d4 lo[2][4], hi[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      lo[m][n] = acc[m][n];
      hi[m][n] = acc[2 + m][n];
    }
  const EpiSums p0 = epilogue_rows<TI, TO, 2>(lo, a, I, J, pos, 0, rowf);
  const EpiSums p1 = epilogue_rows<TI, TO, 2>(hi, a, I, J, pos, 32, rowf);
  if (lane == 0) {
    double *p = a.parts + (int64_t)pos * NPART;
    p[0] = p0.e2 + p1.e2;
    p[1] = p0.tx + p1.tx;
    p[2] = p0.ts + p1.ts;
    p[3] = p0.nr + p1.nr;
    p[4] = (double)nk;
  }
}

}  // namespace

void launch_square_f64_lds(Ctx &c, const TileArgs &a) {
  if (a.ntiles <= 0) return;
  if (a.tb != 2) fail(SP2_ERR_INVALID_ARG, "FP64 LDS-load square: 2 x 2 tiles");
  const bool gen = a.ypool != a.xpool || a.npass != 1 || a.xanti || a.yanti;
  if (gen && !(a.ypool && a.yidxmap && a.ybits && (a.npass == 1 || a.npass == 2)))
    fail(SP2_ERR_INVALID_ARG, "tiled product: incomplete second operand");
  const unsigned g = (unsigned)(8 * a.xcd_chunk);
  if (a.xprec == P32) {
    // FP32-stored operands, FP32 result (the FP64 tail of an expansion whose
    // FP64 iterates do not fit in device memory)
    if (gen || a.full || a.oprec != P32)
      fail(SP2_ERR_INVALID_ARG, "FP64 square of FP32 values: square only, FP32 result");
    k_square_f64_lds<float, float, false><<<g, 256, 0, c.stream>>>(a);
  } else if (a.xprec != P64) {
    fail(SP2_ERR_INVALID_ARG, "FP64 LDS-load square: FP64 or FP32 operands");
  } else if (a.full) {
    if (!(a.ypool && a.yidxmap && a.ybits) || a.npass != 1 || a.xanti || a.yanti || a.oprec != P64)
      fail(SP2_ERR_INVALID_ARG, "general-storage product: one pass, FP64 output, both operands");
    k_square_f64_lds<double, double, true, true><<<g, 256, 0, c.stream>>>(a);
  } else if (a.oprec == P32) {  // FP64 arithmetic, result rounded to FP32 (the correction's commutator)
    if (!gen) fail(SP2_ERR_INVALID_ARG, "FP64 square with FP32 output is for products only");
    k_square_f64_lds<double, float, true><<<g, 256, 0, c.stream>>>(a);
  } else if (gen) {
    k_square_f64_lds<double, double, true><<<g, 256, 0, c.stream>>>(a);
  } else {
    k_square_f64_lds<double, double, false><<<g, 256, 0, c.stream>>>(a);
  }
  SP2_LAUNCH_CHECK();
}

}  // namespace sp2
