// C ABI and driver of the SP2 / SP2ACC density-matrix expansion.
//
// sp2_density follows section "Density matrix construction":
//   Step 1   schedule (host, schedule.h) and X_0 = (lmax I - F) / w with its
//            truncation (Algorithm 1);
//   Step 2   Algorithm 2: per iteration one block-sparse symmetric square of
//            X~_i on MFMA whose epilogue writes X_{i+1} = f_{i+1}(X~_i) and
//            the partial sums of e_i = ||X~_i - X~_i^2||_F and
//            t_i = tr(X~_i - X~_i^2); then the truncation of X_{i+1}; the
//            parameterless stopping test runs on the host on three scalars;
//   Step 3   homo/lumo estimates from e_i and t_i (host).
// The only device -> host traffic per iteration is a handful of scalars and
// the sizes needed to allocate the next pattern.
#include <unistd.h>

#include <chrono>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <limits>

#include "internal.h"
#include "schedule.h"

struct sp2_ctx : public sp2::Ctx {};

namespace sp2 {

namespace {

constexpr double NaN = std::numeric_limits<double>::quiet_NaN();

// per-iteration progress on stderr when SP2_VERBOSE is set (long runs)
bool verbose() {
  static const bool v = [] {
    const char *s = std::getenv("SP2_VERBOSE");
    return s && *s && *s != '0';
  }();
  return v;
}

Buf view(const void *p, size_t bytes) {
  Buf b;
  b.p = const_cast<void *>(p);
  b.bytes = bytes;
  b.ctx = nullptr;  // not owned
  return b;
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ matrices
struct OwnedBsr {
  sp2_bsr pub;
  Buf row_ptr, col_idx, val;
};

void check_input(const sp2_bsr *M, const char *what) {
  if (!M) fail(SP2_ERR_INVALID_ARG, std::string(what) + " is NULL");
  if (M->bs != B) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": block size must be 64");
  if (M->n <= 0) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": n must be positive");
  if (M->nbr != ceil_div(M->n, B)) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": nbr != ceil(n / 64)");
  if (M->nbr > MAX_NBR) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": more than 32768 block rows");
  if (M->nnzb < 0 || M->nnzb > (int64_t)0x7fffffff) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": bad nnzb");
  if (!M->row_ptr || (M->nnzb > 0 && (!M->col_idx || !M->val)))
    fail(SP2_ERR_INVALID_ARG, std::string(what) + ": NULL array");
}

// Borrowed upper BSR -> internal pattern (row_of computed, slot = identity).
// Validates the structure on the device.
// general: the matrix is in general storage (any column 0 <= col < nbr);
// otherwise symmetric upper storage (row <= col)
Pattern borrow_pattern(Ctx &c, const sp2_bsr *M, const char *what, bool general = false) {
  check_input(M, what);
  Pattern p;
  p.n = M->n;
  p.nbr = (int)M->nbr;
  p.nnzb = M->nnzb;
  std::vector<int64_t> rp(p.nbr + 1);
  c.d2h(rp.data(), M->row_ptr, sizeof(int64_t) * (p.nbr + 1));
  if (rp[0] != 0 || rp[p.nbr] != p.nnzb) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": row_ptr ends");
  for (int i = 0; i < p.nbr; ++i)
    if (rp[i + 1] < rp[i]) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": row_ptr not monotone");
  p.row_ptr = view(M->row_ptr, sizeof(int64_t) * (p.nbr + 1));
  p.col_idx = view(M->col_idx, sizeof(int32_t) * p.nnzb);
  p.row_of = c.alloc(sizeof(int32_t) * (p.nnzb > 0 ? p.nnzb : 1));
  launch_row_of(c, M->row_ptr, p.nbr, p.row_of.as<int32_t>());
  Buf flag = c.alloc(sizeof(int32_t));
  launch_fill_i32(c, flag.as<int32_t>(), 1, 0);
  if (general)
    launch_validate_general(c, M->row_ptr, M->col_idx, p.nbr, p.nnzb, flag.as<int32_t>());
  else
    launch_validate_pattern(c, M->row_ptr, M->col_idx, p.nbr, p.nnzb, flag.as<int32_t>());
  int32_t f = 0;
  c.d2h(&f, flag.p, sizeof(f));
  if (f)
    fail(SP2_ERR_INVALID_ARG, std::string(what) + (general ? ": columns must satisfy 0 <= col < nbr, strictly increasing"
                                                           : ": columns must satisfy row <= col < nbr, strictly increasing"));
  return p;
}

void check_finite(Ctx &c, const double *v, int64_t n, const char *what) {
  Buf flag = c.alloc(sizeof(int32_t));
  launch_fill_i32(c, flag.as<int32_t>(), 1, 0);
  launch_check_finite(c, v, n, flag.as<int32_t>());
  int32_t f = 0;
  c.d2h(&f, flag.p, sizeof(f));
  if (f) fail(SP2_ERR_NONFINITE, std::string(what) + " holds non-finite values");
}

Maps build_maps(Ctx &c, const Pattern &p, bool with_adj) {
  Maps m;
  m.nbr = p.nbr;
  m.W = (p.nbr + 31) / 32;
  m.idxmap = c.alloc(sizeof(int32_t) * (size_t)p.nbr * p.nbr);
  m.bits = c.alloc(sizeof(uint32_t) * (size_t)p.nbr * m.W);
  launch_build_maps(c, p.row_of.as<int32_t>(), p.col_idx.as<int32_t>(), p.slot.p ? p.slot.as<int32_t>() : nullptr,
                    p.nnzb, p.nbr, m.W, m.idxmap.as<int32_t>(), m.bits.as<uint32_t>());
  if (with_adj) {
    Buf cnt = c.alloc(sizeof(int64_t) * p.nbr);
    m.adj_ptr = c.alloc(sizeof(int64_t) * (p.nbr + 1));
    launch_popcount_rows(c, m.bits.as<uint32_t>(), p.nbr, m.W, cnt.as<int64_t>());
    scan_exclusive_i64(c, cnt.as<int64_t>(), m.adj_ptr.as<int64_t>(), p.nbr);
    c.d2h(&m.nadj, m.adj_ptr.as<int64_t>() + p.nbr, sizeof(int64_t));
    m.adj_col = c.alloc(sizeof(int32_t) * (m.nadj > 0 ? m.nadj : 1));
    launch_extract_rows(c, m.bits.as<uint32_t>(), p.nbr, m.W, m.adj_ptr.as<int64_t>(), m.adj_col.as<int32_t>(),
                        nullptr);
  }
  return m;
}

// upper block pattern from block-row bitmaps (J >= I bits only), slot = position
Pattern pattern_from_bits(Ctx &c, int64_t n, int nbr, int W, const Buf &outbits) {
  Pattern o;
  o.n = n;
  o.nbr = nbr;
  Buf cnt = c.alloc(sizeof(int64_t) * nbr);
  launch_popcount_rows(c, outbits.as<uint32_t>(), nbr, W, cnt.as<int64_t>());
  o.row_ptr = c.alloc(sizeof(int64_t) * (nbr + 1));
  scan_exclusive_i64(c, cnt.as<int64_t>(), o.row_ptr.as<int64_t>(), nbr);
  c.d2h(&o.nnzb, o.row_ptr.as<int64_t>() + nbr, sizeof(int64_t));
  if (o.nnzb > (int64_t)0x7fffffff) fail(SP2_ERR_INVALID_ARG, "product pattern exceeds 2^31 blocks");
  o.col_idx = c.alloc(sizeof(int32_t) * (o.nnzb > 0 ? o.nnzb : 1));
  o.row_of = c.alloc(sizeof(int32_t) * (o.nnzb > 0 ? o.nnzb : 1));
  launch_extract_rows(c, outbits.as<uint32_t>(), nbr, W, o.row_ptr.as<int64_t>(), o.col_idx.as<int32_t>(),
                      o.row_of.as<int32_t>());
  return o;  // slot empty: identity
}

// block pattern of X^2 (upper blocks), output slot = position
Pattern symbolic_square(Ctx &c, const Pattern &p, const Maps &m) {
  Buf outbits = c.alloc(sizeof(uint32_t) * (size_t)p.nbr * m.W);
  launch_symbolic(c, m.bits.as<uint32_t>(), m.adj_ptr.as<int64_t>(), m.adj_col.as<int32_t>(), p.nbr, m.W,
                  outbits.as<uint32_t>());
  return pattern_from_bits(c, p.n, p.nbr, m.W, outbits);
}

// block pattern of X Y + Y X (upper blocks) for symmetric patterns of X and Y
Pattern symbolic_pair(Ctx &c, int64_t n, const Maps &mx, const Maps &my) {
  Buf outbits = c.alloc(sizeof(uint32_t) * (size_t)mx.nbr * mx.W);
  launch_symbolic(c, my.bits.as<uint32_t>(), mx.adj_ptr.as<int64_t>(), mx.adj_col.as<int32_t>(), mx.nbr, mx.W,
                  outbits.as<uint32_t>(), mx.bits.as<uint32_t>(), my.adj_ptr.as<int64_t>(),
                  my.adj_col.as<int32_t>());
  return pattern_from_bits(c, n, mx.nbr, mx.W, outbits);
}

std::shared_ptr<Pool> new_pool(Ctx &c, int prec, int64_t nslots) {
  auto pl = std::make_shared<Pool>();
  pl->prec = prec;
  pl->nslots = nslots;
  pl->vals = c.alloc((size_t)(nslots > 0 ? nslots : 1) * BB * (prec == P64 ? 8 : 4));
  return pl;
}

const int32_t *slot_ptr(const Pattern &p) { return p.slot.p ? p.slot.as<int32_t>() : nullptr; }

// copy of a pattern (device arrays)
Pattern clone_pattern(Ctx &c, const Pattern &p) {
  Pattern o;
  o.n = p.n;
  o.nbr = p.nbr;
  o.nnzb = p.nnzb;
  const size_t nb = (size_t)(p.nnzb > 0 ? p.nnzb : 1);
  o.row_ptr = c.alloc(sizeof(int64_t) * (p.nbr + 1));
  o.col_idx = c.alloc(sizeof(int32_t) * nb);
  o.row_of = c.alloc(sizeof(int32_t) * nb);
  SP2_HIP(hipMemcpyAsync(o.row_ptr.p, p.row_ptr.p, sizeof(int64_t) * (p.nbr + 1), hipMemcpyDeviceToDevice, c.stream));
  if (p.nnzb > 0) {
    SP2_HIP(hipMemcpyAsync(o.col_idx.p, p.col_idx.p, sizeof(int32_t) * p.nnzb, hipMemcpyDeviceToDevice, c.stream));
    SP2_HIP(hipMemcpyAsync(o.row_of.p, p.row_of.p, sizeof(int32_t) * p.nnzb, hipMemcpyDeviceToDevice, c.stream));
  }
  if (p.slot.p) {
    o.slot = c.alloc(sizeof(int32_t) * nb);
    if (p.nnzb > 0)
      SP2_HIP(hipMemcpyAsync(o.slot.p, p.slot.p, sizeof(int32_t) * p.nnzb, hipMemcpyDeviceToDevice, c.stream));
  }
  return o;
}

// contiguous copy of a matrix in a new pool of precision prec (slot = identity)
DMat compact_values(Ctx &c, const DMat &m, int prec) {
  DMat o;
  o.pat = clone_pattern(c, m.pat);
  o.pat.slot.reset();
  o.pool = new_pool(c, prec, m.pat.nnzb);
  launch_gather(c, m.pool->vals.p, m.pool->prec, slot_ptr(m.pat), m.pat.nnzb, o.pool->vals.p, prec);
  return o;
}

sp2_bsr *export_bsr(Ctx &c, const DMat &m) {
  auto *o = new OwnedBsr();
  o->row_ptr = c.alloc(sizeof(int64_t) * (m.pat.nbr + 1));
  o->col_idx = c.alloc(sizeof(int32_t) * (m.pat.nnzb > 0 ? m.pat.nnzb : 1));
  o->val = c.alloc(sizeof(double) * BB * (size_t)(m.pat.nnzb > 0 ? m.pat.nnzb : 1));
  SP2_HIP(hipMemcpyAsync(o->row_ptr.p, m.pat.row_ptr.p, sizeof(int64_t) * (m.pat.nbr + 1), hipMemcpyDeviceToDevice,
                         c.stream));
  if (m.pat.nnzb > 0)
    SP2_HIP(hipMemcpyAsync(o->col_idx.p, m.pat.col_idx.p, sizeof(int32_t) * m.pat.nnzb, hipMemcpyDeviceToDevice,
                           c.stream));
  launch_gather(c, m.pool->vals.p, m.pool->prec, slot_ptr(m.pat), m.pat.nnzb, o->val.p, P64);
  c.sync();
  o->pub.n = m.pat.n;
  o->pub.bs = B;
  o->pub.owned = 1;
  o->pub.nbr = m.pat.nbr;
  o->pub.nnzb = m.pat.nnzb;
  o->pub.row_ptr = o->row_ptr.as<int64_t>();
  o->pub.col_idx = o->col_idx.as<int32_t>();
  o->pub.val = o->val.as<double>();
  return &o->pub;
}

// borrowed input matrix as an internal DMat (values not copied)
DMat borrow_matrix(Ctx &c, const sp2_bsr *M, const char *what, bool general = false) {
  DMat d;
  d.pat = borrow_pattern(c, M, what, general);
  d.pool = std::make_shared<Pool>();
  d.pool->prec = P64;
  d.pool->nslots = M->nnzb;
  d.pool->vals = view(M->val, sizeof(double) * BB * (size_t)M->nnzb);
  return d;
}

// Truncation and masking keep the pool and drop positions from the pattern; a
// pool left with many unused slots is copied to a contiguous one, so that the
// dropped blocks do not stay resident through the next square (and the BF16x3
// images, packed per slot, cover only the kept blocks).
DMat compact_if_sparse(Ctx &c, DMat X) {
  if (X.pool && X.pat.nnzb < X.pool->nslots - X.pool->nslots / 8) return compact_values(c, X, X.pool->prec);
  return X;
}
// ------------------------------------------------------------------ steps
// BF16x3 operand images of X (32 KB per pool slot), or an empty buffer for the
// other arithmetics
Buf pack_operand(Ctx &c, const DMat &X, int mode) {
  Buf b;
  if (mode != M_BF16X3) return b;
  if (X.pool->prec != P32) fail(SP2_ERR_INVALID_ARG, "BF16x3 operands must hold FP32 values");
  b = c.alloc((size_t)(X.pool->nslots > 0 ? X.pool->nslots : 1) * BB * 4 * sizeof(uint16_t));
  launch_pack_bf16x3(c, X.pool->vals.as<float>(), slot_ptr(X.pat), X.pat.nnzb, b.as<uint16_t>());
  return b;
}

// Tile edge of a BF16x3 product: 4 x 4 output tiles (k_square_tile4_bf16x3,
// half the operand traffic per block product) once the output pattern holds
// at least 35% of the upper blocks, else 2 x 2 (the 4 x 4 K scan runs over the
// union of 8 block rows, wasteful on sparse patterns; on the C1 expansion the
// two kernels break even near 35-40%).  The environment variable
// SP2_BF16X3_TILE = 2 or 4 forces one of them.
int tile_edge(int mode, int64_t nout, int nbr) {
  if (mode != M_BF16X3) return 2;
  if (const char *e = std::getenv("SP2_BF16X3_TILE")) {
    if (e[0] == '2') return 2;
    if (e[0] == '4') return 4;
  }
  return (double)nout >= 0.35 * 0.5 * (double)nbr * (double)(nbr + 1) ? 4 : 2;
}

// FP64 squares and products run k_square_f64_lds (operands loaded straight
// to LDS, bit-identical to k_square_tile, also for FP32-stored operands);
// SP2_F64_KERNEL=tile in the environment selects k_square_tile instead.
bool use_f64_lds() {
  const char *e = std::getenv("SP2_F64_KERNEL");
  return !(e && e[0] == 't');
}

struct SquareOut {
  DMat next;      // X_{i+1} (or S when fused == false) on the square's pattern
  Buf parts;      // nout x NPART
  double sums[NPART];
  double kernel_s = 0.0;  // device time of the MFMA square (HIP events)
  double plan_s = 0.0;    // with SP2_VERBOSE: wall time of planning, allocation and packing before the kernel
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    SP2_HIP(hipEventCreate(&a));
    SP2_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

SquareOut square_step(Ctx &c, const DMat &X, const Maps &m, int mode, int oprec, double ca, double cb, double cc) {
  const auto t0 = std::chrono::steady_clock::now();
  SquareOut r;
  r.next.pat = symbolic_square(c, X.pat, m);
  const int64_t nout = r.next.pat.nnzb;
  r.next.pool = new_pool(c, oprec, nout);
  r.parts = c.alloc(sizeof(double) * NPART * (size_t)(nout > 0 ? nout : 1));
  // output tiles over the square's pattern
  Maps om = build_maps(c, r.next.pat, false);
  Buf tiles;
  const int tb = tile_edge(mode, nout, X.pat.nbr);
  const int64_t ntiles = build_tiles(c, om.idxmap.as<int32_t>(), X.pat.nbr, tiles, tb);
  TileArgs ta;
  ta.tb = tb;
  ta.xpool = X.pool->vals.p;
  ta.xprec = X.pool->prec;
  ta.idxmap = m.idxmap.as<int32_t>();
  ta.bits = m.bits.as<uint32_t>();
  ta.ypool = ta.xpool;
  ta.yidxmap = ta.idxmap;
  ta.ybits = ta.bits;
  ta.gpool = ta.xpool;
  ta.gidxmap = ta.idxmap;
  Buf xpack = pack_operand(c, X, mode);
  ta.xpack = xpack.p;
  ta.ypack = xpack.p;
  ta.nbr = X.pat.nbr;
  ta.W = m.W;
  ta.oidx = om.idxmap.as<int32_t>();
  ta.tiles = tiles.as<int32_t>();
  ta.ntiles = ntiles;
  ta.xcd_chunk = (ntiles + 7) / 8;
  ta.opool = r.next.pool->vals.p;
  ta.oprec = oprec;
  ta.ca = ca;
  ta.cb = cb;
  ta.cc = cc;
  ta.n = X.pat.n;
  ta.parts = r.parts.as<double>();
  EventPair ev;
  if (verbose()) {
    c.sync();
    r.plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  SP2_HIP(hipEventRecord(ev.a, c.stream));
  if (mode == M_F64 && tb == 2 && use_f64_lds())
    launch_square_f64_lds(c, ta);
  else
    launch_square_tile(c, mode, ta);
  SP2_HIP(hipEventRecord(ev.b, c.stream));
  Buf sums = c.alloc(sizeof(double) * NPART);
  launch_reduce_parts(c, ta.parts, nout, NPART, sums.as<double>());
  c.d2h(r.sums, sums.p, sizeof(double) * NPART);
  float ms = 0.0f;
  SP2_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  r.kernel_s = 1e-3 * (double)ms;
  c.kern_s[mode] += r.kernel_s;
  c.kern_flops[mode] += r.sums[4] * 2.0 * B * B * B;
  if (nout > 0) c.kern_launches[mode]++;
  return r;
}

// Options of a two-operand product (the tiled kernel's general mode)
struct PairOpt {
  bool neg2 = false;             // X Y - Y X instead of X Y + Y X
  bool yanti = false;            // Y antisymmetric (upper blocks stored)
  const DMat *G = nullptr;       // matrix of the cb term
  const Maps *mg = nullptr;
  double ca = 0.0, cb = 0.0, cc = 1.0;
  int mode = M_F64, oprec = P64;
  const Pattern *outpat = nullptr;  // output pattern; default the block pattern of X Y + Y X
};

// out = ca I + cb G + cc (X Y +- Y X) on upper blocks.  X, Y (and G) hold
// values in the precision the mode multiplies (FP64 or FP32); the maps need
// adjacency lists when the output pattern is the product's own.
SquareOut pair_product(Ctx &c, const DMat &X, const Maps &mx, const DMat &Y, const Maps &my, const PairOpt &po) {
  const auto t0 = std::chrono::steady_clock::now();
  const int need = po.mode == M_F64 ? P64 : P32;
  if (po.mode == M_F64 && po.oprec == P32 && po.G) fail(SP2_ERR_INVALID_ARG, "pair product: FP32 output takes no G");
  if (X.pool->prec != need || Y.pool->prec != need || (po.G && po.G->pool->prec != need))
    fail(SP2_ERR_INVALID_ARG, "pair product: operand precision does not match the arithmetic");
  if (X.pat.nbr != Y.pat.nbr) fail(SP2_ERR_INVALID_ARG, "pair product: operand sizes differ");
  SquareOut r;
  if (po.outpat) {
    r.next.pat = clone_pattern(c, *po.outpat);
    r.next.pat.slot.reset();
  } else {
    r.next.pat = symbolic_pair(c, X.pat.n, mx, my);
  }
  const int64_t nout = r.next.pat.nnzb;
  r.next.pool = new_pool(c, po.oprec, nout);
  r.parts = c.alloc(sizeof(double) * NPART * (size_t)(nout > 0 ? nout : 1));
  Maps om = build_maps(c, r.next.pat, false);
  Buf tiles;
  const int tb = tile_edge(po.mode, nout, X.pat.nbr);
  const int64_t ntiles = build_tiles(c, om.idxmap.as<int32_t>(), X.pat.nbr, tiles, tb);
  TileArgs ta;
  ta.tb = tb;
  ta.xpool = X.pool->vals.p;
  ta.xprec = X.pool->prec;
  ta.idxmap = mx.idxmap.as<int32_t>();
  ta.bits = mx.bits.as<uint32_t>();
  ta.ypool = Y.pool->vals.p;
  ta.yidxmap = my.idxmap.as<int32_t>();
  ta.ybits = my.bits.as<uint32_t>();
  Buf xpack = pack_operand(c, X, po.mode), ypack = pack_operand(c, Y, po.mode);
  ta.xpack = xpack.p;
  ta.ypack = ypack.p;
  ta.npass = 2;
  ta.neg2 = po.neg2 ? 1 : 0;
  ta.xanti = 0;
  ta.yanti = po.yanti ? 1 : 0;
  ta.gpool = po.G ? po.G->pool->vals.p : nullptr;
  ta.gidxmap = po.G ? po.mg->idxmap.as<int32_t>() : nullptr;
  ta.nbr = X.pat.nbr;
  ta.W = mx.W;
  ta.oidx = om.idxmap.as<int32_t>();
  ta.tiles = tiles.as<int32_t>();
  ta.ntiles = ntiles;
  ta.xcd_chunk = (ntiles + 7) / 8;
  ta.opool = r.next.pool->vals.p;
  ta.oprec = po.oprec;
  ta.ca = po.ca;
  ta.cb = po.cb;
  ta.cc = po.cc;
  ta.n = X.pat.n;
  ta.parts = r.parts.as<double>();
  EventPair ev;
  if (verbose()) {
    c.sync();
    r.plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  SP2_HIP(hipEventRecord(ev.a, c.stream));
  if (po.mode == M_F64 && tb == 2 && use_f64_lds())
    launch_square_f64_lds(c, ta);
  else
    launch_square_tile(c, po.mode, ta);
  SP2_HIP(hipEventRecord(ev.b, c.stream));
  Buf sums = c.alloc(sizeof(double) * NPART);
  launch_reduce_parts(c, ta.parts, nout, NPART, sums.as<double>());
  c.d2h(r.sums, sums.p, sizeof(double) * NPART);
  float ms = 0.0f;
  SP2_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  r.kernel_s = 1e-3 * (double)ms;
  c.kern_s[po.mode] += r.kernel_s;
  c.kern_flops[po.mode] += r.sums[4] * 2.0 * B * B * B;
  if (nout > 0) c.kern_launches[po.mode]++;
  return r;
}

// a A + b B in FP64 on the union of the two block patterns
DMat add_union(Ctx &c, const DMat &A, double a, const DMat &Bm, double b) {
  Maps ma = build_maps(c, A.pat, false), mb = build_maps(c, Bm.pat, false);
  Buf ub = c.alloc(sizeof(uint32_t) * (size_t)ma.nbr * ma.W);
  launch_or_upper(c, ma.bits.as<uint32_t>(), mb.bits.as<uint32_t>(), ma.nbr, ma.W, ub.as<uint32_t>());
  DMat o;
  o.pat = pattern_from_bits(c, A.pat.n, ma.nbr, ma.W, ub);
  o.pool = new_pool(c, P64, o.pat.nnzb);
  launch_add_union(c, o.pat.row_of.as<int32_t>(), o.pat.col_idx.as<int32_t>(), o.pat.nnzb, ma.nbr, A.pool->vals.p,
                   A.pool->prec, ma.idxmap.as<int32_t>(), a, Bm.pool->vals.p, Bm.pool->prec,
                   mb.idxmap.as<int32_t>(), b, o.pool->vals.as<double>());
  return o;
}

// ------------------------------------------------------- general storage
// Block map and bitmaps of a general pattern (of its transpose with
// transpose), adjacency lists of the bitmap rows with with_adj.
Maps build_maps_general(Ctx &c, const Pattern &p, bool transpose, bool with_idx, bool with_adj) {
  Maps m;
  m.nbr = p.nbr;
  m.W = (p.nbr + 31) / 32;
  if (with_idx) m.idxmap = c.alloc(sizeof(int32_t) * (size_t)p.nbr * p.nbr);
  m.bits = c.alloc(sizeof(uint32_t) * (size_t)p.nbr * m.W);
  launch_build_maps_general(c, p.row_of.as<int32_t>(), p.col_idx.as<int32_t>(), slot_ptr(p), p.nnzb, p.nbr, m.W,
                            transpose, with_idx ? m.idxmap.as<int32_t>() : nullptr, m.bits.as<uint32_t>());
  if (with_adj) {
    Buf cnt = c.alloc(sizeof(int64_t) * p.nbr);
    m.adj_ptr = c.alloc(sizeof(int64_t) * (p.nbr + 1));
    launch_popcount_rows(c, m.bits.as<uint32_t>(), p.nbr, m.W, cnt.as<int64_t>());
    scan_exclusive_i64(c, cnt.as<int64_t>(), m.adj_ptr.as<int64_t>(), p.nbr);
    c.d2h(&m.nadj, m.adj_ptr.as<int64_t>() + p.nbr, sizeof(int64_t));
    m.adj_col = c.alloc(sizeof(int32_t) * (m.nadj > 0 ? m.nadj : 1));
    launch_extract_rows(c, m.bits.as<uint32_t>(), p.nbr, m.W, m.adj_ptr.as<int64_t>(), m.adj_col.as<int32_t>(),
                        nullptr);
  }
  return m;
}

// out = ca I + cb G + cc A B for A, B (and G) in general storage, on the block
// pattern of A B joined with G's and, when ca != 0, the diagonal; output in
// general storage.  mode M_F64 (FP64 operands) or M_BF16X3 (FP32 operands).
SquareOut general_product(Ctx &c, const DMat &A, const DMat &Bm, const DMat *G, double ca, double cb, double cc,
                          int mode) {
  const auto t0 = std::chrono::steady_clock::now();
  const int need = mode == M_F64 ? P64 : P32;
  if (mode != M_F64 && mode != M_BF16X3) fail(SP2_ERR_INVALID_ARG, "general product: FP64 or BF16x3 arithmetic");
  if (A.pool->prec != need || Bm.pool->prec != need || (G && G->pool->prec != need))
    fail(SP2_ERR_INVALID_ARG, "general product: operand precision does not match the arithmetic");
  if (A.pat.nbr != Bm.pat.nbr || A.pat.n != Bm.pat.n || (G && G->pat.n != A.pat.n))
    fail(SP2_ERR_INVALID_ARG, "general product: operand sizes differ");
  const int nbr = A.pat.nbr;
  Maps ma = build_maps_general(c, A.pat, false, true, true);   // rows I of A: K lists, slots
  Maps mbr = build_maps_general(c, Bm.pat, false, false, false);  // rows K of B (symbolic)
  Maps mbt = build_maps_general(c, Bm.pat, true, true, false);   // columns J of B: K bits, slots
  Maps mg;
  if (G) mg = build_maps_general(c, G->pat, false, true, false);
  SquareOut r;
  {
    Buf outbits = c.alloc(sizeof(uint32_t) * (size_t)nbr * ma.W);
    launch_symbolic(c, mbr.bits.as<uint32_t>(), ma.adj_ptr.as<int64_t>(), ma.adj_col.as<int32_t>(), nbr, ma.W,
                    outbits.as<uint32_t>(), nullptr, nullptr, nullptr, false);
    launch_or_general(c, outbits.as<uint32_t>(), G ? mg.bits.as<uint32_t>() : nullptr, nbr, ma.W, ca != 0.0);
    r.next.pat = pattern_from_bits(c, A.pat.n, nbr, ma.W, outbits);
  }
  const int64_t nout = r.next.pat.nnzb;
  const int oprec = mode == M_F64 ? P64 : P32;
  r.next.pool = new_pool(c, oprec, nout);
  r.parts = c.alloc(sizeof(double) * NPART * (size_t)(nout > 0 ? nout : 1));
  Maps om = build_maps_general(c, r.next.pat, false, true, false);
  Buf tiles;
  // the 4 x 4 BF16x3 tiles pay off at the same density as in the symmetric
  // square (there counted over the upper triangle)
  const int tb = tile_edge(mode, nout / 2, nbr);
  const int64_t ntiles = build_tiles(c, om.idxmap.as<int32_t>(), nbr, tiles, tb, true);
  TileArgs ta;
  ta.tb = tb;
  ta.full = 1;
  ta.xpool = A.pool->vals.p;
  ta.xprec = A.pool->prec;
  ta.idxmap = ma.idxmap.as<int32_t>();
  ta.bits = ma.bits.as<uint32_t>();
  ta.ypool = Bm.pool->vals.p;
  ta.yidxmap = mbt.idxmap.as<int32_t>();
  ta.ybits = mbt.bits.as<uint32_t>();
  Buf xpack = pack_operand(c, A, mode), ypack = pack_operand(c, Bm, mode);
  ta.xpack = xpack.p;
  ta.ypack = ypack.p;
  ta.npass = 1;
  ta.gpool = G ? G->pool->vals.p : nullptr;
  ta.gidxmap = G ? mg.idxmap.as<int32_t>() : nullptr;
  ta.nbr = nbr;
  ta.W = ma.W;
  ta.oidx = om.idxmap.as<int32_t>();
  ta.tiles = tiles.as<int32_t>();
  ta.ntiles = ntiles;
  ta.xcd_chunk = (ntiles + 7) / 8;
  ta.opool = r.next.pool->vals.p;
  ta.oprec = oprec;
  ta.ca = ca;
  ta.cb = cb;
  ta.cc = cc;
  ta.n = A.pat.n;
  ta.parts = r.parts.as<double>();
  EventPair ev;
  if (verbose()) {
    c.sync();
    r.plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  SP2_HIP(hipEventRecord(ev.a, c.stream));
  if (mode == M_F64)
    launch_square_f64_lds(c, ta);
  else
    launch_square_tile_bf16x3(c, ta);
  SP2_HIP(hipEventRecord(ev.b, c.stream));
  Buf sums = c.alloc(sizeof(double) * NPART);
  launch_reduce_parts(c, ta.parts, nout, NPART, sums.as<double>());
  c.d2h(r.sums, sums.p, sizeof(double) * NPART);
  float ms = 0.0f;
  SP2_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  r.kernel_s = 1e-3 * (double)ms;
  c.kern_s[mode] += r.kernel_s;
  c.kern_flops[mode] += r.sums[4] * 2.0 * B * B * B;
  if (nout > 0) c.kern_launches[mode]++;
  return r;
}

// general storage of a symmetric upper-BSR matrix (FP64)
DMat expand_upper(Ctx &c, const DMat &U) {
  if (U.pool->prec != P64) fail(SP2_ERR_INVALID_ARG, "expand_upper: FP64 values");
  Maps m = build_maps(c, U.pat, false);  // symmetric: both orientations of every stored block
  DMat o;
  o.pat = pattern_from_bits(c, U.pat.n, m.nbr, m.W, m.bits);
  o.pool = new_pool(c, P64, o.pat.nnzb);
  launch_expand_upper(c, o.pat.row_of.as<int32_t>(), o.pat.col_idx.as<int32_t>(), o.pat.nnzb, m.nbr,
                      m.idxmap.as<int32_t>(), U.pool->vals.as<double>(), o.pool->vals.as<double>());
  return o;
}

struct TruncResult {
  double err_frob = 0.0, err_mixed = 0.0;
  int64_t removed = 0;
};

// truncate in place (pattern replaced; pool untouched)
TruncResult truncate_matrix(Ctx &c, DMat &X, const double *nrm2, double tau, int norm, int64_t coarse_bs) {
  TruncResult res;
  if (norm == SP2_TRUNC_NONE || !(tau > 0.0)) return res;
  Buf keep = c.alloc(sizeof(int64_t) * (X.pat.nnzb > 0 ? X.pat.nnzb : 1));
  TruncOut to;
  int nc = 1;
  truncate_select(c, X.pat, nrm2, tau, norm, coarse_bs, keep.as<int64_t>(), to, &nc);
  res.removed = to.removed;
  if (to.removed > 0) {
    Pattern np;
    if (!X.pat.slot.p) {  // identity slots: materialise before compaction
      X.pat.slot = c.alloc(sizeof(int32_t) * (X.pat.nnzb > 0 ? X.pat.nnzb : 1));
      launch_iota_i32(c, X.pat.slot.as<int32_t>(), X.pat.nnzb);
    }
    compact_pattern(c, X.pat, keep.as<int64_t>(), np);
    X.pat = std::move(np);
  }
  // error norms of E from the per-segment removed sums
  if (norm == SP2_TRUNC_FROB) {
    const double s = to.seg_err.empty() ? 0.0 : to.seg_err[0];
    res.err_frob = std::sqrt(s);
    res.err_mixed = res.err_frob;
  } else if (!to.seg_err.empty()) {
    double f2 = 0.0, mx = 0.0;
    for (int R = 0; R < nc; ++R) {
      double row = 0.0;
      for (int S = 0; S < nc; ++S) {
        const double v = (R <= S) ? to.seg_err[(size_t)R * nc + S] : to.seg_err[(size_t)S * nc + R];
        row += std::sqrt(v);
        if (R == S)
          f2 += v;
        else if (R < S)
          f2 += 2.0 * v;
      }
      mx = std::fmax(mx, row);
    }
    res.err_frob = std::sqrt(f2);
    res.err_mixed = mx;
  }
  return res;
}

Buf column(Ctx &c, const Buf &parts, int64_t nrows, int col);

}  // namespace

}  // namespace sp2

// column extraction kernel (strided partial sums -> contiguous)
namespace sp2 {
namespace {
__global__ void k_col(const double *parts, int64_t nrows, int ncols, int col, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nrows) out[i] = parts[i * ncols + col];
}
Buf column(Ctx &c, const Buf &parts, int64_t nrows, int col) {
  Buf o = c.alloc(sizeof(double) * (nrows > 0 ? nrows : 1));
  if (nrows > 0) {
    k_col<<<(unsigned)((nrows + 255) / 256), 256, 0, c.stream>>>(parts.as<double>(), nrows, NPART, col,
                                                                 o.as<double>());
    SP2_LAUNCH_CHECK();
  }
  return o;
}
}  // namespace
}  // namespace sp2


// ====================================================================== driver
namespace sp2 {

namespace {

__global__ void k_scale(double *v, int64_t n, double s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] *= s;
}
void scale_pool(Ctx &c, double *v, int64_t n, double s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  k_scale<<<(unsigned)g, 256, 0, c.stream>>>(v, n, s);
  SP2_LAUNCH_CHECK();
}

// X_0 = (lmax I - F) / w on F's pattern plus the diagonal blocks (Algorithm 1)
DMat init_x0(Ctx &c, const DMat &F, double lmax, double w) {
  const int nbr = F.pat.nbr;
  Buf cnt = c.alloc(sizeof(int64_t) * nbr);
  launch_diag_missing(c, F.pat.row_ptr.as<int64_t>(), F.pat.col_idx.as<int32_t>(), nbr, cnt.as<int64_t>());
  DMat X;
  X.pat.n = F.pat.n;
  X.pat.nbr = nbr;
  X.pat.row_ptr = c.alloc(sizeof(int64_t) * (nbr + 1));
  scan_exclusive_i64(c, cnt.as<int64_t>(), X.pat.row_ptr.as<int64_t>(), nbr);
  c.d2h(&X.pat.nnzb, X.pat.row_ptr.as<int64_t>() + nbr, sizeof(int64_t));
  const int64_t nn = X.pat.nnzb;
  X.pat.col_idx = c.alloc(sizeof(int32_t) * nn);
  X.pat.row_of = c.alloc(sizeof(int32_t) * nn);
  Buf src = c.alloc(sizeof(int32_t) * nn);
  launch_x0_pattern(c, F.pat.row_ptr.as<int64_t>(), F.pat.col_idx.as<int32_t>(), nbr, X.pat.row_ptr.as<int64_t>(),
                    X.pat.col_idx.as<int32_t>(), src.as<int32_t>());
  launch_row_of(c, X.pat.row_ptr.as<int64_t>(), nbr, X.pat.row_of.as<int32_t>());
  X.pool = new_pool(c, P64, nn);
  launch_init_x0(c, F.pool->vals.as<double>(), src.as<int32_t>(), X.pat.row_of.as<int32_t>(),
                 X.pat.col_idx.as<int32_t>(), nn, F.pat.n, lmax, w, X.pool->vals.as<double>());
  return X;
}

Buf norms_of(Ctx &c, const DMat &X) {
  Buf nrm2 = c.alloc(sizeof(double) * (X.pat.nnzb > 0 ? X.pat.nnzb : 1));
  launch_block_norms(c, X.pool->vals.p, X.pool->prec, slot_ptr(X.pat), X.pat.nnzb, nrm2.as<double>());
  return nrm2;
}

// make the stored diagonal blocks of X exactly symmetric (sign 1) or
// antisymmetric (sign -1); X must own its pool
void sym_diag(Ctx &c, DMat &X, double sign) {
  launch_sym_diag(c, X.pool->vals.p, X.pool->prec, X.pat.row_ptr.as<int64_t>(), X.pat.col_idx.as<int32_t>(),
                  slot_ptr(X.pat), X.pat.nbr, sign);
}

// ||X||_F of the whole symmetric (or antisymmetric) matrix held by its upper blocks
double frob_norm(Ctx &c, const DMat &X) {
  if (X.pat.nnzb <= 0) return 0.0;
  Buf nrm2 = norms_of(c, X);
  launch_weight_offdiag(c, nrm2.as<double>(), X.pat.row_of.as<int32_t>(), X.pat.col_idx.as<int32_t>(), X.pat.nnzb);
  Buf sum = c.alloc(sizeof(double));
  launch_reduce_parts(c, nrm2.as<double>(), X.pat.nnzb, 1, sum.as<double>());
  double v = 0.0;
  c.d2h(&v, sum.p, sizeof(double));
  return std::sqrt(std::fmax(v, 0.0));
}

// restrict X to the blocks present in mask (pattern + slots rewritten)
void restrict_to(Ctx &c, DMat &X, const Pattern &mask) {
  Maps mm = build_maps(c, mask, false);
  Buf keep = c.alloc(sizeof(int64_t) * (X.pat.nnzb > 0 ? X.pat.nnzb : 1));
  launch_mark_in_mask(c, X.pat, mm.bits.as<uint32_t>(), mm.W, keep.as<int64_t>());
  if (!X.pat.slot.p) {
    X.pat.slot = c.alloc(sizeof(int32_t) * (X.pat.nnzb > 0 ? X.pat.nnzb : 1));
    launch_iota_i32(c, X.pat.slot.as<int32_t>(), X.pat.nnzb);
  }
  Pattern np;
  compact_pattern(c, X.pat, keep.as<int64_t>(), np);
  X.pat = std::move(np);
}

// a low-precision square resolves e down to about ten times its rounding noise
double low_floor(int mode, double trX) { return 10.0 * e_noise(mode, trX); }

}  // namespace

// Values of an iterate kept in pinned host memory.  The device -> host copy
// runs on the context's copy stream while the main stream goes on with the
// square of the same iterate; the device pool is held until the copy has
// completed (wait()).
struct HostCopy {
  Pattern pat;                 // device pattern of the iterate (slots included)
  int prec = P32;
  int64_t nslots = 0;
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t ready = nullptr;  // the values are complete on the main stream
  hipEvent_t done = nullptr;   // the device -> host copy has completed
  std::shared_ptr<Pool> src;   // the device pool until the copy completed
  void wait() {
    if (src && done) (void)hipEventSynchronize(done);
    src.reset();
  }
  ~HostCopy() {
    if (done) (void)hipEventSynchronize(done);
    src.reset();
    if (host) (void)hipHostFree(host);
    if (ready) (void)hipEventDestroy(ready);
    if (done) (void)hipEventDestroy(done);
  }
};

struct TapeIter {
  Pattern mask;                  // block pattern of X~_i
  int p = -1;                    // polynomial that produced X_i (i >= 1)
  double alpha = 1.0, ca = 0.0, cb = 0.0, cc = 0.0;
  int mode = M_F64;              // arithmetic of the square of X~_i
  int prec = P64;                // storage precision of X~_i
  std::shared_ptr<DMat> ckpt;    // compact copy of X~_i, or empty
  std::shared_ptr<HostCopy> hcopy;  // copy of X~_i in pinned host memory, or empty
};

struct Tape {
  Ctx *ctx = nullptr;
  int64_t n = 0, n_occ = 0;
  double lmax = 0.0, w = 1.0;
  int n_iter = 0, n_ckpt = 0;
  int64_t bytes = 0;
  int adj_mode = -1;  // arithmetic of adjoint steps at low-precision iterations (-1: as recorded)
  std::vector<TapeIter> it;
  int step_mode(int i) const { return (adj_mode >= 0 && it[i].mode != M_F64) ? adj_mode : it[i].mode; }
};

}  // namespace sp2

struct sp2_tape : public sp2::Tape {};

namespace sp2 {
namespace {

// X with values in precision prec: a view sharing the pool when it already is
DMat as_prec(Ctx &c, const DMat &X, int prec) {
  if (X.pool->prec == prec) {
    DMat d;
    d.pat = clone_pattern(c, X.pat);
    d.pool = X.pool;
    return d;
  }
  return compact_values(c, X, prec);
}

struct CorrStats {
  int rounds = 0;
  double time_s = 0.0, flops = 0.0, delta_norm = 0.0, step_norm = 0.0, e_last = 0.0;
  int64_t max_nnzb = 0;
};

DMat replay_step(Ctx &c, const Tape &t, int i, const DMat &Xprev);
DMat checkpoint_copy(const Tape &t, int i);

void add_checkpoint(Ctx &c, Tape &t, int i, const DMat &X) {
  auto d = std::make_shared<DMat>(compact_values(c, X, X.pool->prec));
  t.bytes += (int64_t)d->pat.nnzb * BB * (d->pool->prec == P64 ? 8 : 4);
  t.it[i].ckpt = d;
  t.n_ckpt++;
}

constexpr double FL_BLOCK = 2.0 * B * B * B;  // flops of one 64 x 64 x 64 block product

int64_t available_host_bytes() {
  const long pages = sysconf(_SC_AVPHYS_PAGES), psz = sysconf(_SC_PAGESIZE);
  return (pages > 0 && psz > 0) ? (int64_t)pages * (int64_t)psz : 0;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// One density-matrix expansion as a resumable computation.  begin() runs
// Step 1 and Algorithm 1 (schedule, X_0 and its truncation); each step() runs
// one iteration of Algorithm 2 (square with the fused update, e_i and t_i,
// the stopping test, truncation of X_{i+1}) or, after the expansion, one
// product of the subspace correction; finish() runs Step 3 and returns D.
struct Solver {
  Ctx &c;
  // ---- problem
  DMat F;  // borrowed
  int64_t N = 0, n_occ = 0;
  double lmin = 0.0, lmax = 0.0, w = 1.0;
  sp2_options o{};
  int lowmode = M_F64;
  bool corr = false, low_to_end = false;
  bool low_started = false;  // the low-precision squares have begun
  bool tail32 = false;       // FP64-arithmetic tail on FP32-stored iterates (tail_storage = 1)
  Sched sch;
  int n_max = 0;
  // ---- adjoint tape
  std::unique_ptr<sp2_tape> tape;
  int ck_every = 1;
  int64_t tape_budget = 0;
  // ---- expansion
  DMat X;  // X~_i (after the expansion: the current D)
  int i = 0;
  std::vector<double> e, t, trv, errF, errM, itime, iflops, ksq, alph{1.0}, taus;
  std::vector<int> p{-1}, precv;
  std::vector<char> stor32v;  // X~_i stored in FP32
  std::vector<int64_t> nnzbv;
  int switch_iter = -1, n = -1, stop_reason = 0, status = SP2_OK;
  bool criterion_seen = false;  // the stopping test was evaluated at an admissible iteration
  double alg_flops = 0.0;
  int64_t max_nnzb = 0, seq_bytes = 0;
  // ---- iterates recorded for the correction (masks, polynomials, a prefix of copies)
  Tape ct;
  int64_t seq_budget = 0;
  bool seq_full = false;
  int64_t host_budget = 0, host_bytes = 0;
  bool host_full = false;
  int n_recomputed = 0;
  std::vector<std::shared_ptr<HostCopy>> pending;  // host copies still holding their device pools
  int pf_k = -1;                                   // iterate being prefetched from host memory
  DMat pf_X;
  hipEvent_t pf_ready = nullptr, pf_done = nullptr;
  // ---- correction state
  enum Phase { EXPAND, CORRECT, FINISHED, FAILED };
  enum CStage { C_COMM, C_DELTA, C_DERIV, C_PURIFY };
  Phase phase = EXPAND;
  CStage cstage = C_COMM;
  int cround = 0, ck = 0, csub = 0, n_deriv = 0;
  double beta = 1e-9, deriv_tol = 1e-3;
  DMat C, dX, Xi, Rm;
  CorrStats cs;
  // ---- accounting
  double busy_s = 0.0;     // time spent inside begin / step / finish
  double last_flops = 0.0; // algorithmic flops of the last step
  sp2_step_info info{};    // facts of the last step

  explicit Solver(Ctx &ctx) : c(ctx) {}
  ~Solver();
  void begin(const sp2_bsr *Fin, int64_t n_occ_, double lmin_, double lmax_, const double *hub, const double *llb,
             const sp2_options &opt);
  bool step();
  int finish(sp2_bsr **D_out, double *hest, double *lest, sp2_stats *st, sp2_tape **tape_out);

 private:
  void iterate();
  void record_iterate(int mode);
  std::shared_ptr<HostCopy> host_store(const DMat &M);
  DMat host_load(const HostCopy &h);
  void correct_step();
  void note(const DMat &M) { cs.max_nnzb = std::max(cs.max_nnzb, M.pat.nnzb); }
  // the low precision may square X~_k (its gap image has reached low_start_xi)
  bool low_begins(int k) const {
    return !sch.bounds || !(o.low_start_xi > 0.0) || k >= (int)sch.xi.size() || sch.xi[k] >= o.low_start_xi;
  }
  // blocks of a correction intermediate dropped within the Frobenius budget beta
  void drop(DMat &M, const SquareOut &so) {
    note(M);
    Buf nrm2 = column(c, so.parts, M.pat.nnzb, 3);
    truncate_matrix(c, M, nrm2.as<double>(), beta, SP2_TRUNC_FROB, o.coarse_bs);
  }
};

void Solver::begin(const sp2_bsr *Fin, int64_t n_occ_, double lmin_, double lmax_, const double *hub,
                   const double *llb, const sp2_options &opt) {
  auto t0 = std::chrono::steady_clock::now();
  o = opt;
  n_occ = n_occ_;
  lmin = lmin_;
  lmax = lmax_;
  // ---- argument checks ---------------------------------------------------------
  check_input(Fin, "F");
  N = Fin->n;
  if (!(n_occ > 0 && n_occ < N)) fail(SP2_ERR_INVALID_ARG, "n_occ must lie in (0, n)");
  if (!(std::isfinite(lmin) && std::isfinite(lmax) && lmin < lmax))
    fail(SP2_ERR_INVALID_ARG, "need finite lmin < lmax");
  if ((hub == nullptr) != (llb == nullptr)) fail(SP2_ERR_INVALID_ARG, "give both homo/lumo bounds or neither");
  if (hub && !(lmin <= *hub && *hub < *llb && *llb <= lmax))
    fail(SP2_ERR_BAD_BOUNDS, "bounds must satisfy lmin <= homo_ub < lumo_lb <= lmax");
  if (o.precision < 0 || o.precision > 2) fail(SP2_ERR_INVALID_ARG, "unknown precision");
  if (o.trunc_norm < 0 || o.trunc_norm > 2) fail(SP2_ERR_INVALID_ARG, "unknown truncation norm");
  if (o.n_max_cap < 1 || o.n_max_cap > 1000) fail(SP2_ERR_INVALID_ARG, "n_max_cap must be in [1, 1000]");
  if (o.trunc_norm == SP2_TRUNC_FROBINF && (o.coarse_bs <= 0 || o.coarse_bs % B))
    fail(SP2_ERR_INVALID_ARG, "coarse_bs must be a positive multiple of 64");
  if (!(o.gamma >= 0.0) || !(o.tau_fixed >= 0.0) || std::isnan(o.switch_tol) || !(o.idem_stop >= 0.0))
    fail(SP2_ERR_INVALID_ARG, "tolerances must be >= 0 (switch_tol: any number)");
  if (o.correct < 0 || o.correct > 8) fail(SP2_ERR_INVALID_ARG, "correct must be in [0, 8]");
  if (o.correct > 0 && (o.corr_purify < 1 || o.corr_purify > 16))
    fail(SP2_ERR_INVALID_ARG, "corr_purify must be in [1, 16]");
  if (!(o.corr_tol >= 0.0)) fail(SP2_ERR_INVALID_ARG, "corr_tol must be >= 0");
  if (o.corr_mem < 0) fail(SP2_ERR_INVALID_ARG, "corr_mem must be >= 0");
  if (o.adjoint_precision < -1 || o.adjoint_precision > 2) fail(SP2_ERR_INVALID_ARG, "unknown adjoint_precision");
  if (!(o.low_start_xi >= 0.0 && o.low_start_xi < 1.0)) fail(SP2_ERR_INVALID_ARG, "low_start_xi must be in [0, 1)");
  if (o.tail_storage != 0 && o.tail_storage != 1) fail(SP2_ERR_INVALID_ARG, "tail_storage must be 0 or 1");
  if (o.low_floor_stop != 0 && o.low_floor_stop != 1) fail(SP2_ERR_INVALID_ARG, "low_floor_stop must be 0 or 1");
  if (o.tail_storage == 1 && o.correct > 0)
    fail(SP2_ERR_INVALID_ARG, "tail_storage = 1 is not combined with the subspace correction");
  lowmode = o.precision == SP2_PREC_FP32 ? M_F32 : (o.precision == SP2_PREC_BF16X3 ? M_BF16X3 : M_F64);
  corr = o.correct > 0;
  // with the correction and no switch tolerance, or with a negative one, the
  // whole expansion stays in the low precision and stops by its own criterion
  low_to_end = (corr && !(o.switch_tol > 0.0)) || o.switch_tol < 0.0;
  beta = o.corr_tol > 0.0 ? o.corr_tol : 1e-9;

  c.peak_bytes = c.live_bytes;
  F = borrow_matrix(c, Fin, "F");
  check_finite(c, Fin->val, Fin->nnzb * (int64_t)BB, "F");

  // ---- Step 1 ---------------------------------------------------------------------
  w = lmax - lmin;
  sch = hub ? make_schedule(lmin, lmax, *hub, *llb, o.accel != 0, o.gamma, o.tau_fixed, o.n_max_cap)
            : make_tc2(lmin, lmax, o.tau_fixed, o.n_max_cap);
  n_max = sch.n_max;

  if (o.record_tape) {
    tape.reset(new sp2_tape());
    tape->ctx = &c;
    tape->n = N;
    tape->n_occ = n_occ;
    tape->lmax = lmax;
    tape->w = w;
    tape->adj_mode = o.adjoint_precision < 0 ? -1
                     : (o.adjoint_precision == SP2_PREC_FP64 ? M_F64
                        : (o.adjoint_precision == SP2_PREC_FP32 ? M_F32 : M_BF16X3));
    const int nck = o.n_checkpoints > 0 ? o.n_checkpoints : (int)std::ceil(std::sqrt((double)(n_max + 1)));
    ck_every = std::max(1, (int)std::ceil((double)(n_max + 1) / (double)nck));
    size_t fr = 0, tot = 0;
    SP2_HIP(hipMemGetInfo(&fr, &tot));
    tape_budget = (int64_t)std::min(0.2 * (double)tot, 0.3 * (double)fr);
  }

  // ---- Algorithm 1 ------------------------------------------------------------------
  X = init_x0(c, F, lmax, w);
  {
    Buf nrm2 = norms_of(c, X);
    TruncResult tr = truncate_matrix(c, X, nrm2.as<double>(), sch.tau[0], o.trunc_norm, o.coarse_bs);
    errF.push_back(tr.err_frob);
    errM.push_back(tr.err_mixed);
    taus.push_back(sch.tau[0]);
  }
  if (lowmode != M_F64 && low_begins(0)) {
    X = compact_values(c, X, P32);
    low_started = true;
  }
  switch_iter = lowmode != M_F64 ? -1 : 0;

  if (corr) {
    size_t fr = 0, tot = 0;
    SP2_HIP(hipMemGetInfo(&fr, &tot));
    seq_budget = o.corr_mem > 0 ? o.corr_mem : (int64_t)std::min(0.25 * (double)tot, 0.35 * (double)fr);
    host_budget = o.corr_host_mem > 0 ? o.corr_host_mem
                  : (o.corr_host_mem < 0 ? 0 : (int64_t)(0.75 * (double)available_host_bytes()));
    deriv_tol = o.corr_deriv_tol > 0.0 ? o.corr_deriv_tol : 1e-2;
    SP2_HIP(hipEventCreateWithFlags(&pf_ready, hipEventDisableTiming));
    SP2_HIP(hipEventCreateWithFlags(&pf_done, hipEventDisableTiming));
    ct.ctx = &c;
    ct.n = N;
    ct.lmax = lmax;
    ct.w = w;
  }
  c.sync();
  busy_s += seconds_since(t0);
}

Solver::~Solver() {
  // no copy on the second stream may outlive the buffers it reads or writes
  if (pf_done) (void)hipStreamWaitEvent(c.stream, pf_done, 0);
  if (c.copy_stream) (void)hipStreamSynchronize(c.copy_stream);
  pf_X = DMat();
  pending.clear();
  ct.it.clear();
  if (pf_ready) (void)hipEventDestroy(pf_ready);
  if (pf_done) (void)hipEventDestroy(pf_done);
}

// X~_i for the correction: its mask and polynomial, and a copy on the device
// (while corr_mem lasts), in pinned host memory (while corr_host_mem lasts)
// or none (recomputed from the previous iterate when needed)
void Solver::record_iterate(int mode) {
  // copies started in earlier iterations ran under their own squares: they
  // have completed, and their device pools can go
  for (auto &h : pending) h->wait();
  pending.clear();
  ct.it.emplace_back();
  TapeIter &ti = ct.it.back();
  ti.mask = clone_pattern(c, X.pat);
  ti.mask.slot.reset();
  ti.mode = mode;
  ti.prec = X.pool->prec;
  if (i >= 1) {
    ti.p = p[i];
    ti.alpha = alph[i];
    poly_coeffs(p[i], alph[i], ti.ca, ti.cb, ti.cc);
  }
  // the derivative steps stop before the first X~_k (k >= 1) with e_k below
  // corr_deriv_tol: once one has been seen, later iterates are never used
  for (int k = 1; k < i; ++k)
    if (e[k] < deriv_tol) return;
  const int64_t esz = X.pool->prec == P64 ? 8 : 4;
  const int64_t bytes = X.pat.nnzb * (int64_t)BB * esz;
  if (i == 0 || (!seq_full && seq_bytes + bytes <= seq_budget)) {
    add_checkpoint(c, ct, i, X);
    seq_bytes += bytes;
    return;
  }
  seq_full = true;
  const int64_t hb = X.pool->nslots * (int64_t)BB * esz;
  if (!host_full && host_bytes + hb <= host_budget) {
    if (auto h = host_store(X)) {
      ti.hcopy = h;
      host_bytes += hb;
      pending.push_back(h);
      return;
    }
  }
  host_full = true;
}

// start copying the value pool of M to pinned host memory on the copy stream
// (after the work already queued on the main stream); null when the host
// allocation fails
std::shared_ptr<HostCopy> Solver::host_store(const DMat &M) {
  auto h = std::make_shared<HostCopy>();
  h->prec = M.pool->prec;
  h->nslots = M.pool->nslots;
  h->bytes = (size_t)std::max<int64_t>(M.pool->nslots, 1) * BB * (h->prec == P64 ? 8 : 4);
  if (hipHostMalloc(&h->host, h->bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    h->host = nullptr;
    return nullptr;
  }
  h->pat = clone_pattern(c, M.pat);
  hipStream_t cs = c.copies();
  SP2_HIP(hipEventCreateWithFlags(&h->ready, hipEventDisableTiming));
  SP2_HIP(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  SP2_HIP(hipEventRecord(h->ready, c.stream));
  SP2_HIP(hipStreamWaitEvent(cs, h->ready, 0));
  SP2_HIP(hipMemcpyAsync(h->host, M.pool->vals.p, h->bytes, hipMemcpyDeviceToHost, cs));
  SP2_HIP(hipEventRecord(h->done, cs));
  h->src = M.pool;
  return h;
}

// device copy of a host-stored iterate; the host -> device copy runs on the
// copy stream and pf_done marks its completion (the main stream must wait on
// it before the values are used)
DMat Solver::host_load(const HostCopy &h) {
  DMat d;
  d.pat = clone_pattern(c, h.pat);
  d.pool = new_pool(c, h.prec, h.nslots);
  hipStream_t cs = c.copies();
  SP2_HIP(hipEventRecord(pf_ready, c.stream));  // earlier users of the new buffer are done
  SP2_HIP(hipStreamWaitEvent(cs, pf_ready, 0));
  SP2_HIP(hipMemcpyAsync(d.pool->vals.p, h.host, h.bytes, hipMemcpyHostToDevice, cs));
  SP2_HIP(hipEventRecord(pf_done, cs));
  return d;
}

// one iteration of Algorithm 2
void Solver::iterate() {
  auto t_it = std::chrono::steady_clock::now();
  const int mode = (X.pool->prec == P32 && !tail32) ? lowmode : M_F64;
  if (tape) {
    tape->it.emplace_back();
    TapeIter &ti = tape->it.back();
    ti.mask = clone_pattern(c, X.pat);
    ti.mask.slot.reset();
    ti.mode = mode;
    ti.prec = X.pool->prec;
    if (i >= 1) {
      ti.p = p[i];
      ti.alpha = alph[i];
      poly_coeffs(p[i], alph[i], ti.ca, ti.cb, ti.cc);
    }
    const int64_t ckb = X.pat.nnzb * (int64_t)BB * (X.pool->prec == P64 ? 8 : 4);
    if (i % ck_every == 0 && (i == 0 || tape->bytes + ckb <= tape_budget)) add_checkpoint(c, *tape, i, X);
  }
  if (corr) record_iterate(mode);
  nnzbv.push_back(X.pat.nnzb);
  max_nnzb = std::max(max_nnzb, X.pat.nnzb);
  precv.push_back(mode == M_F64 ? SP2_PREC_FP64 : o.precision);
  stor32v.push_back(X.pool->prec == P32 ? 1 : 0);

  Maps m = build_maps(c, X.pat, true);
  const bool have_next = i < n_max;
  double ca = 0.0, cb = 0.0, cc = 1.0;
  if (sch.bounds && have_next) poly_coeffs(sch.p[i + 1], sch.alpha[i + 1], ca, cb, cc);
  SquareOut so = square_step(c, X, m, mode, X.pool->prec, ca, cb, cc);
  const double ei = std::sqrt(std::fmax(so.sums[0], 0.0));
  const double trX = so.sums[1], trS = so.sums[2];
  e.push_back(ei);
  t.push_back(trX - trS);
  trv.push_back(trX);
  const double fl = so.sums[4] * FL_BLOCK;
  iflops.push_back(fl);
  ksq.push_back(so.kernel_s);
  alg_flops += fl;
  last_flops = fl;

  // ---- stopping test (Algorithm 2) -----------------------------------------
  // the criterion compares e_i with e_{i-2}: both from FP64 squares, the
  // older one of an iterate the FP64 tail has already squared once (the
  // first FP64 iterates still carry the low-precision rounding, which two
  // FP64 squares remove; stopping on it would end at the low-precision floor)
  bool stop = false;
  const bool fp64_window = mode == M_F64 && (switch_iter >= 0 && i >= switch_iter + 2);
  const bool low_window = low_to_end && mode != M_F64;
  const bool admissible = i >= std::max(sch.n_min, 2) && p[i] != p[i - 1];
  if (i >= 1 && (fp64_window || low_window)) {
    if (admissible) criterion_seen = true;
    if (admissible && e[i] > C_STOP * e[i - 2] * e[i - 2]) {
      stop = true;
      stop_reason = SP2_STOP_CRITERION;
    } else if (o.idem_stop > 0.0 && e[i] <= o.idem_stop) {
      stop = true;
      stop_reason = SP2_STOP_IDEMPOTENCY;
    } else if (low_window && o.low_floor_stop && i >= 2 && ei < low_floor(mode, trX)) {
      // the low-precision squares cannot resolve e below this level: the
      // next iterates would only repeat it until the criterion fires
      stop = true;
      stop_reason = SP2_STOP_NOISE_FLOOR;
    }
  }
  if (!stop && i == n_max) {
    stop = true;
    stop_reason = SP2_STOP_NMAX;
    // a warning when the criterion could have fired and did not; an FP64
    // tail that reaches n_max before its first admissible test ends where
    // the schedule (valid bounds) places convergence
    if (criterion_seen || switch_iter <= 0) status = SP2_WARN_NOT_CONVERGED;
  }
  if (stop) {
    n = i;
    if (corr) ct.it.pop_back();  // the correction replays X~_0 .. X~_{n-1}
    c.sync();
    itime.push_back(seconds_since(t_it));
    phase = corr ? CORRECT : FINISHED;
    return;
  }

  // ---- next polynomial and truncation of X_{i+1} ----------------------------------
  int pn;
  double an;
  if (sch.bounds) {
    pn = sch.p[i + 1];
    an = sch.alpha[i + 1];
  } else {
    pn = std::fabs(trS - (double)n_occ) < std::fabs(2.0 * trX - trS - (double)n_occ) ? 1 : 0;
    an = 1.0;
    poly_coeffs(pn, an, ca, cb, cc);
    launch_update(c, X.pool->vals.p, X.pool->prec, m.idxmap.as<int32_t>(), X.pat.nbr,
                  so.next.pat.row_of.as<int32_t>(), so.next.pat.col_idx.as<int32_t>(), so.next.pat.nnzb,
                  so.next.pool->vals.p, so.next.pool->prec, ca, cb, cc, N, so.parts.as<double>());
  }
  p.push_back(pn);
  alph.push_back(an);
  DMat Xn = std::move(so.next);
  const int64_t nout = Xn.pat.nnzb;
  X = DMat{};  // X~_i is not needed any more: release it before X_{i+1} is compacted
  {
    Buf nrm2 = column(c, so.parts, nout, 3);
    TruncResult tr = truncate_matrix(c, Xn, nrm2.as<double>(), sch.tau[i + 1], o.trunc_norm, o.coarse_bs);
    errF.push_back(tr.err_frob);
    errM.push_back(tr.err_mixed);
    taus.push_back(sch.tau[i + 1]);
  }
  const bool to_fp64 = (o.switch_tol > 0.0 && ei < o.switch_tol) || (!low_to_end && ei < low_floor(mode, trX));
  if (Xn.pool->prec == P32 && to_fp64 && !tail32 && o.tail_storage == 1) {
    // the FP64 tail keeps the FP32 storage: only the arithmetic changes
    tail32 = true;
    switch_iter = i + 1;
    Xn = compact_if_sparse(c, std::move(Xn));
  } else if (Xn.pool->prec == P32 && to_fp64 && !tail32) {
    Xn = compact_values(c, Xn, P64);
    sym_diag(c, Xn, 1.0);  // the FP64 tail starts from the symmetric part
    switch_iter = i + 1;
  } else if (lowmode != M_F64 && !low_started && switch_iter < 0) {
    // FP64 squares while the gap image is narrow; the low precision from the
    // first X~_i whose gap reaches low_start_xi, unless e_i already calls for
    // the FP64 tail (the run then stays in FP64)
    if (o.switch_tol > 0.0 && ei < o.switch_tol) {
      switch_iter = 0;
      Xn = compact_if_sparse(c, std::move(Xn));
    } else if (low_begins(i + 1)) {
      Xn = compact_values(c, Xn, P32);
      low_started = true;
    } else {
      Xn = compact_if_sparse(c, std::move(Xn));
    }
  } else {
    Xn = compact_if_sparse(c, std::move(Xn));
  }
  X = std::move(Xn);
  c.sync();
  itime.push_back(seconds_since(t_it));
  if (verbose())
    std::fprintf(stderr, "[sp2] iter %d p=%d alpha=%.6f nnzb=%lld e=%.3e t=%.3e square %.1f ms (%.2f TFLOP/s)%s\n", i,
                 p[i], alph[i], (long long)nnzbv[i], e[i], t[i], 1e3 * ksq[i],
                 ksq[i] > 0.0 ? iflops[i] / ksq[i] / 1e12 : 0.0, mode == M_F64 ? "" : " low precision");
  ++i;
}

// One product of the occupied-subspace correction (the operation documented
// with sp2_options.correct): Delta = [D, [D, F]], dD = J Delta along the
// stored X~_0 .. X~_{n-1} (derivative of the polynomial steps, blocks dropped
// within corr_tol), D <- FP64 purification of D + dD.  The commutator
// C = [D, F] is formed in FP64 (it is small: the difference of two O(1)
// products); [D, C] and the derivative steps use the arithmetic the expansion
// used for each X~_i.
void Solver::correct_step() {
  const int lp = lowmode == M_F64 ? P64 : P32;
  last_flops = 0.0;
  switch (cstage) {
    case C_COMM: {
      if (cround == 0) {
        // Once an iterate is close to a projector P (e_i small), the remaining
        // derivative steps map dX to P dX (I - P) + (I - P) dX P plus parts
        // inside the two subspaces, which the purification removes: they
        // change the correction only at relative order e_i and are skipped.
        n_deriv = n;
        for (int k = 1; k < n; ++k)
          if (e[k] < deriv_tol) {
            n_deriv = k;
            break;
          }
        for (auto &h : pending) h->wait();
        pending.clear();
        // the symmetric part of D: a low-precision iterate's diagonal blocks
        // carry antisymmetric rounding noise, which the correction must not see
        X = compact_values(c, X, X.pool->prec);
        sym_diag(c, X, 1.0);
      }
      // C = D F - F D, antisymmetric, in FP64 arithmetic (stored in the low
      // precision: the cancellation happens in the accumulators)
      DMat D64 = as_prec(c, X, P64);
      Maps mD = build_maps(c, D64.pat, true), mF = build_maps(c, F.pat, true);
      PairOpt pc;
      pc.neg2 = true;
      pc.oprec = lp;
      SquareOut co = pair_product(c, D64, mD, F, mF, pc);
      last_flops = co.sums[4] * FL_BLOCK;
      C = std::move(co.next);
      sym_diag(c, C, -1.0);
      drop(C, co);
      if (verbose())
        std::fprintf(stderr, "[sp2] correction: C = [D, F] nnzb=%lld square %.1f ms\n", (long long)C.pat.nnzb,
                     1e3 * co.kernel_s);
      cstage = C_DELTA;
      break;
    }
    case C_DELTA: {
      // dX~_0 = -(D C - C D) / w = -Delta / w
      DMat Dl = as_prec(c, X, lp), Cl = as_prec(c, C, lp);
      C = DMat();
      Maps mD = build_maps(c, Dl.pat, true), mC = build_maps(c, Cl.pat, true);
      PairOpt pd;
      pd.neg2 = true;
      pd.yanti = true;
      pd.cc = -1.0 / w;
      pd.mode = lowmode;
      pd.oprec = lp;
      SquareOut dd = pair_product(c, Dl, mD, Cl, mC, pd);
      last_flops = dd.sums[4] * FL_BLOCK;
      cs.delta_norm = std::sqrt(std::fmax(dd.sums[0], 0.0));  // no G: sums[0] = ||D C - C D||_F^2
      dX = std::move(dd.next);
      drop(dX, dd);
      if (verbose())
        std::fprintf(stderr, "[sp2] correction: Delta nnzb=%lld ||Delta||=%.3e product %.1f ms\n",
                     (long long)dX.pat.nnzb, cs.delta_norm, 1e3 * dd.kernel_s);
      ck = 0;
      cstage = C_DERIV;
      break;
    }
    case C_DERIV: {
      // derivative of X_{k+1} = ca I + cb X~_k + cc X~_k^2 along dX~_k
      const int k = ck;
      const auto t_step = std::chrono::steady_clock::now();
      TapeIter &tk = ct.it[k];
      const char *src = "";
      if (tk.ckpt) {
        Xi = checkpoint_copy(ct, k);
      } else if (pf_k == k) {
        SP2_HIP(hipStreamWaitEvent(c.stream, pf_done, 0));
        Xi = std::move(pf_X);
        pf_k = -1;
        src = " (host copy)";
      } else if (tk.hcopy) {
        Xi = host_load(*tk.hcopy);
        SP2_HIP(hipStreamWaitEvent(c.stream, pf_done, 0));
        src = " (host copy)";
      } else {
        Xi = replay_step(c, ct, k, Xi);
        ++n_recomputed;
        src = " (recomputed iterate)";
      }
      if (verbose()) c.sync();
      const double t_it = seconds_since(t_step);
      if (cround == o.correct - 1) {  // the last round needs X~_k only here
        tk.ckpt.reset();
        tk.hcopy.reset();
      }
      // the next host-stored iterate comes back under this step's product
      if (k + 1 < n_deriv && !ct.it[k + 1].ckpt && ct.it[k + 1].hcopy) {
        pf_X = host_load(*ct.it[k + 1].hcopy);
        pf_k = k + 1;
      }
      const int mi = Xi.pool->prec == P32 ? lowmode : M_F64;
      DMat G = as_prec(c, dX, Xi.pool->prec);
      Maps mX = build_maps(c, Xi.pat, true), mG = build_maps(c, G.pat, true);
      double ca, cb, cc;
      poly_coeffs(p[k + 1], alph[k + 1], ca, cb, cc);
      PairOpt pj;
      pj.G = &G;
      pj.mg = &mG;
      pj.cb = cb;
      pj.cc = cc;
      pj.mode = mi;
      pj.oprec = Xi.pool->prec;
      SquareOut jo = pair_product(c, Xi, mX, G, mG, pj);
      last_flops = jo.sums[4] * FL_BLOCK;
      dX = std::move(jo.next);
      drop(dX, jo);
      if (verbose())
        std::fprintf(stderr, "[sp2] correction: derivative step %d/%d nnzb=%lld%s product %.1f ms (planning %.1f ms), "
                     "iterate %.1f ms, step %.1f ms\n", k + 1, n_deriv, (long long)dX.pat.nnzb, src, 1e3 * jo.kernel_s,
                     1e3 * jo.plan_s, 1e3 * t_it, 1e3 * seconds_since(t_step));
      ++ck;
      break;
    }
    case C_PURIFY: {
      if (o.corr_mcweeny && csub == 0) {
        // S = P^2 in FP64, written as R = S - P by the square's epilogue; R is
        // small, so its low-precision copy loses nothing the target can see
        Maps m = build_maps(c, X.pat, true);
        SquareOut so = square_step(c, X, m, M_F64, P64, 0.0, -1.0, 1.0);
        last_flops = so.sums[4] * FL_BLOCK;
        cs.e_last = std::sqrt(std::fmax(so.sums[0], 0.0));
        note(so.next);
        Rm = compact_values(c, so.next, lp);
        if (verbose())
          std::fprintf(stderr, "[sp2] correction: McWeeny %d: R = P^2 - P, e=%.3e square %.1f ms\n", ck, cs.e_last,
                       1e3 * so.kernel_s);
        csub = 1;
        break;
      }
      if (o.corr_mcweeny) {
        // P' = 3 P^2 - 2 P^3 = P + R - (P R + R P), the product in the low arithmetic
        SquareOut to;
        {
          DMat Pl = as_prec(c, X, lp);
          Maps mP = build_maps(c, Pl.pat, true), mR = build_maps(c, Rm.pat, true);
          PairOpt pt;
          pt.mode = lowmode;
          pt.oprec = lp;
          to = pair_product(c, Pl, mP, Rm, mR, pt);
        }
        last_flops = to.sums[4] * FL_BLOCK;
        note(to.next);
        DMat PR = add_union(c, X, 1.0, Rm, 1.0);
        Rm = DMat();
        X = DMat();
        X = add_union(c, PR, 1.0, to.next, -1.0);
        PR = DMat();
        to = SquareOut();
        Buf nrm2 = norms_of(c, X);
        truncate_matrix(c, X, nrm2.as<double>(), taus[n], o.trunc_norm, o.coarse_bs);
        if (verbose()) std::fprintf(stderr, "[sp2] correction: McWeeny %d: P' = P + R - (P R + R P)\n", ck);
        csub = 0;
        ++ck;
        if (ck == o.corr_purify) {
          cs.rounds++;
          cround++;
          cstage = C_COMM;
          if (cround == o.correct) phase = FINISHED;
        }
        break;
      }
      double ca, cb, cc;
      poly_coeffs(ck % 2 == 0 ? 1 : 0, 1.0, ca, cb, cc);
      Maps m = build_maps(c, X.pat, true);
      SquareOut so = square_step(c, X, m, M_F64, P64, ca, cb, cc);
      last_flops = so.sums[4] * FL_BLOCK;
      cs.e_last = std::sqrt(std::fmax(so.sums[0], 0.0));
      DMat Pn = std::move(so.next);
      note(Pn);
      Buf nrm2 = column(c, so.parts, Pn.pat.nnzb, 3);
      truncate_matrix(c, Pn, nrm2.as<double>(), taus[n], o.trunc_norm, o.coarse_bs);
      X = std::move(Pn);
      if (verbose())
        std::fprintf(stderr, "[sp2] correction: purification %d e=%.3e square %.1f ms\n", ck, cs.e_last,
                     1e3 * so.kernel_s);
      ++ck;
      if (ck == o.corr_purify) {
        cs.rounds++;
        cround++;
        cstage = C_COMM;
        if (cround == o.correct) phase = FINISHED;
      }
      break;
    }
  }
  if (cstage == C_DERIV && ck == n_deriv) {
    // D + dD, then the purification
    Xi = DMat();
    cs.step_norm = frob_norm(c, dX);
    X = add_union(c, X, 1.0, dX, 1.0);
    dX = DMat();
    note(X);
    ck = 0;
    cstage = C_PURIFY;
  }
  alg_flops += last_flops;
  cs.flops += last_flops;
}

bool Solver::step() {
  if (phase == FINISHED) fail(SP2_ERR_INVALID_ARG, "the expansion has finished: call sp2_density_end");
  if (phase == FAILED) fail(SP2_ERR_INVALID_ARG, "an earlier step failed; release the solver");
  auto t0 = std::chrono::steady_clock::now();
  double ks0[3], kf0[3];
  int64_t kl0[3];
  for (int m = 0; m < 3; ++m) {
    ks0[m] = c.kern_s[m];
    kf0[m] = c.kern_flops[m];
    kl0[m] = c.kern_launches[m];
  }
  const bool expanding = phase == EXPAND;
  const int it0 = i;
  try {
    if (expanding)
      iterate();
    else
      correct_step();
    c.sync();
  } catch (...) {
    phase = FAILED;
    throw;
  }
  const double dt = seconds_since(t0);
  busy_s += dt;
  info = sp2_step_info{};
  info.kind = expanding ? SP2_STEP_ITERATION : SP2_STEP_CORRECTION;
  info.iteration = expanding ? it0 : -1;
  info.flops = last_flops;
  info.wall_s = dt;
  int dom = 0;
  for (int m = 0; m < 3; ++m) {
    info.kernel_s[m] = c.kern_s[m] - ks0[m];
    info.kernel_flops[m] = c.kern_flops[m] - kf0[m];
    info.kernel_launches[m] = (int32_t)(c.kern_launches[m] - kl0[m]);
    if (info.kernel_flops[m] > info.kernel_flops[dom]) dom = m;
  }
  info.precision = dom == M_F64 ? SP2_PREC_FP64 : (dom == M_F32 ? SP2_PREC_FP32 : SP2_PREC_BF16X3);
  if (phase == CORRECT || (phase == FINISHED && corr)) cs.time_s += dt;
  if (phase == FINISHED && corr) {
    ct.it.clear();
    if (verbose())
      std::fprintf(stderr, "[sp2] correction: %d round(s) %.3f s ||Delta||=%.3e ||dD||=%.3e e_last=%.3e\n", cs.rounds,
                   cs.time_s, cs.delta_norm, cs.step_norm, cs.e_last);
  }
  info.done = phase == FINISHED ? 1 : 0;
  return phase == FINISHED;
}

int Solver::finish(sp2_bsr **D_out, double *hest, double *lest, sp2_stats *st, sp2_tape **tape_out) {
  if (phase != FINISHED) fail(SP2_ERR_INVALID_ARG, "the expansion has not finished");
  auto t0 = std::chrono::steady_clock::now();
  // ---- Step 3 and outputs ---------------------------------------------------------
  double h = NaN, l = NaN;
  {
    std::vector<double> noise(n + 1);
    for (int k = 0; k <= n; ++k)
      noise[k] = precv[k] == SP2_PREC_FP64
                     ? (stor32v[k] ? e_noise_fp32_storage(trv[k]) : 0.0)
                     : e_noise(precv[k] == SP2_PREC_FP32 ? M_F32 : M_BF16X3, trv[k]);
    homo_lumo(sch, e, trv, p, alph, n, lmin, lmax, N, n_occ, h, l, &noise);
  }
  double bound = NaN;
  if (sch.bounds) {
    bound = 0.0;
    for (int k = 0; k <= n; ++k)
      if (errM[k] > 0.0) bound += errM[k] / (sch.xi[k] - errM[k]);
  }
  if (status == SP2_OK && std::fabs(trv[n] - (double)n_occ) > 0.5) status = SP2_WARN_TRACE;
  if (X.pool->prec == P32) {  // a low-precision result: return its symmetric part
    X = compact_values(c, X, P32);
    sym_diag(c, X, 1.0);
  }
  *D_out = export_bsr(c, X);
  X = DMat();
  busy_s += seconds_since(t0);
  if (verbose())
    std::fprintf(stderr, "[sp2] %.3f s in the library; device allocator: %lld allocations %.3f s, %lld frees %.3f s "
                 "(context totals)\n", busy_s, (long long)c.n_raw_alloc, c.raw_alloc_s, (long long)c.n_raw_free,
                 c.raw_free_s);
  if (hest) *hest = h;
  if (lest) *lest = l;
  if (st) {
    st->n_iter = n;
    st->n_max = n_max;
    st->n_min = sch.n_min;
    st->stop_reason = stop_reason;
    st->switch_iter = switch_iter;
    st->homo_ub_est = h;
    st->lumo_lb_est = l;
    st->subspace_err_bound = bound;
    st->time_s = busy_s;
    st->alg_flops = alg_flops;
    st->max_nnzb = max_nnzb;
    st->square_time_total_s = 0.0;
    for (int k = 0; k <= n; ++k) st->square_time_total_s += ksq[k];
    st->corr_rounds = cs.rounds;
    st->corr_time_s = cs.time_s;
    st->corr_flops = cs.flops;
    st->corr_delta_norm = cs.delta_norm;
    st->corr_step_norm = cs.step_norm;
    st->corr_e_last = cs.e_last;
    st->corr_max_nnzb = cs.max_nnzb;
    st->seq_bytes = seq_bytes;
    st->seq_host_bytes = host_bytes;
    st->corr_recomputed = n_recomputed;
    st->device_peak_bytes = (int64_t)c.peak_bytes;
    for (int k = 0; k <= n; ++k) {
      if (st->square_time_s) st->square_time_s[k] = ksq[k];
      if (st->e) st->e[k] = e[k];
      if (st->t) st->t[k] = t[k];
      if (st->trace) st->trace[k] = trv[k];
      if (st->alpha) st->alpha[k] = alph[k];
      if (st->tau) st->tau[k] = taus[k];
      if (st->trunc_err_frob) st->trunc_err_frob[k] = errF[k];
      if (st->trunc_err_mixed) st->trunc_err_mixed[k] = errM[k];
      if (st->iter_time_s) st->iter_time_s[k] = itime[k];
      if (st->iter_flops) st->iter_flops[k] = iflops[k];
      if (st->p) st->p[k] = p[k];
      if (st->precision) st->precision[k] = precv[k];
      if (st->nnzb) st->nnzb[k] = nnzbv[k];
    }
  }
  if (tape && tape_out) {
    tape->n_iter = n;
    tape->it.resize(n + 1);
    *tape_out = tape.release();
  }
  return status;
}

int run_density(Ctx &c, const sp2_bsr *Fin, int64_t n_occ, double lmin, double lmax, const double *hub,
                const double *llb, const sp2_options &o, sp2_bsr **D_out, double *hest, double *lest,
                sp2_stats *st, sp2_tape **tape_out) {
  if (!D_out) fail(SP2_ERR_INVALID_ARG, "D_out is NULL");
  *D_out = nullptr;
  if (tape_out) *tape_out = nullptr;
  if (st && st->capacity < o.n_max_cap + 1) fail(SP2_ERR_INVALID_ARG, "stats capacity < n_max_cap + 1");
  if (tape_out && !o.record_tape) fail(SP2_ERR_INVALID_ARG, "a tape needs record_tape = 1");
  Solver s(c);
  s.begin(Fin, n_occ, lmin, lmax, hub, llb, o);
  while (!s.step()) {
  }
  return s.finish(D_out, hest, lest, st, tape_out);
}

}  // namespace

struct SolverHandle {
  Ctx *ctx = nullptr;
  std::unique_ptr<Solver> s;
};

}  // namespace sp2

struct sp2_solver : public sp2::SolverHandle {};

namespace sp2 {
namespace {

// ---------------------------------------------------------------- adjoint
// X~_{i} from X~_{i-1} with the recorded polynomial and mask (frozen map)
DMat replay_step(Ctx &c, const Tape &t, int i, const DMat &Xprev) {
  const TapeIter &ti = t.it[i];
  const TapeIter &tp = t.it[i - 1];
  Maps m = build_maps(c, Xprev.pat, true);
  SquareOut so = square_step(c, Xprev, m, tp.mode, Xprev.pool->prec, ti.ca, ti.cb, ti.cc);
  DMat Xn = std::move(so.next);
  restrict_to(c, Xn, ti.mask);
  if (Xn.pool->prec != ti.prec) {
    // the switch to the FP64 tail: the forward continues from the symmetric part
    Xn = compact_values(c, Xn, ti.prec);
    if (ti.prec == P64) sym_diag(c, Xn, 1.0);
    return Xn;
  }
  return compact_if_sparse(c, std::move(Xn));
}

DMat checkpoint_copy(const Tape &t, int i) {
  DMat d;
  const DMat &ck = *t.it[i].ckpt;
  Ctx &c = *t.ctx;
  d.pat = clone_pattern(c, ck.pat);
  d.pool = ck.pool;  // shared, read-only
  return d;
}


// out = cb G + cc (G X + X G) on the pattern outpat, in the arithmetic of mode
// (FP64, or FP32 values for the FP32 / BF16x3 products)
DMat anticommutator(Ctx &c, const DMat &Gin, const DMat &Xin, const Pattern &outpat, double cb, double cc, int mode) {
  const int prec = mode == M_F64 ? P64 : P32;
  DMat G = as_prec(c, Gin, prec), X = as_prec(c, Xin, prec);
  Maps mg = build_maps(c, G.pat, false), mx = build_maps(c, X.pat, false);
  PairOpt po;
  po.G = &G;
  po.mg = &mg;
  po.cb = cb;
  po.cc = cc;
  po.mode = mode;
  po.oprec = prec;
  po.outpat = &outpat;
  return std::move(pair_product(c, X, mx, G, mg, po).next);
}

void check_same_n(const Tape &t, const sp2_bsr *M, const char *what) {
  check_input(M, what);
  if (M->n != t.n) fail(SP2_ERR_INVALID_ARG, std::string(what) + ": dimension differs from the recorded run");
}

sp2_bsr *run_vjp(Ctx &c, const Tape &t, const sp2_bsr *Win) {
  check_same_n(t, Win, "W");
  DMat W = borrow_matrix(c, Win, "W");
  check_finite(c, Win->val, Win->nnzb * (int64_t)BB, "W");
  const int n = t.n_iter;
  DMat Xbar = std::move(W);
  restrict_to(c, Xbar, t.it[n].mask);  // G_n = M_n o W
  // X~_{i-1} for i = n..1: from the nearest checkpoint or kept replayed iterate
  // below it, replaying forward; replayed iterates are kept (to serve the
  // following, lower i) while they fit in a share of the device memory, else
  // recomputed when needed again
  size_t fr = 0, tot = 0;
  SP2_HIP(hipMemGetInfo(&fr, &tot));
  const int64_t budget = (int64_t)std::min(0.2 * (double)tot, 0.3 * (double)fr);
  std::map<int, DMat> kept;
  int64_t kept_bytes = 0;
  auto bytes_of = [](const DMat &M) { return M.pat.nnzb * (int64_t)BB * (M.pool->prec == P64 ? 8 : 4); };
  auto iterate = [&](int k) -> DMat {
    int b = k;
    while (b > 0 && !t.it[b].ckpt && !kept.count(b)) --b;
    DMat X = kept.count(b) ? as_prec(c, kept[b], kept[b].pool->prec) : checkpoint_copy(t, b);
    for (int j = b + 1; j <= k; ++j) {
      X = replay_step(c, t, j, X);
      const int64_t nb = bytes_of(X);
      if (j < k && kept_bytes + nb <= budget) {
        kept[j] = as_prec(c, X, X.pool->prec);
        kept_bytes += nb;
      }
    }
    return X;
  };
  for (int i = n; i >= 1; --i) {
    DMat X = iterate(i - 1);
    const TapeIter &ti = t.it[i];
    Xbar = anticommutator(c, Xbar, X, t.it[i - 1].mask, ti.cb, ti.cc, t.step_mode(i - 1));
    if (verbose()) std::fprintf(stderr, "[sp2] vjp: step %d nnzb=%lld\n", i, (long long)Xbar.pat.nnzb);
    // iterates at or above i - 1 are not needed any more
    for (auto it = kept.lower_bound(i - 1); it != kept.end();) {
      kept_bytes -= bytes_of(it->second);
      it = kept.erase(it);
    }
  }
  // Fbar = -(M_0 o Xbar) / w  (Xbar already lives on M_0)
  DMat Fb = compact_values(c, Xbar, P64);
  scale_pool(c, Fb.pool->vals.as<double>(), Fb.pat.nnzb * (int64_t)BB, -1.0 / t.w);
  return export_bsr(c, Fb);
}

sp2_bsr *run_jvp(Ctx &c, const Tape &t, const sp2_bsr *dFin) {
  check_same_n(t, dFin, "dF");
  DMat dF = borrow_matrix(c, dFin, "dF");
  check_finite(c, dFin->val, dFin->nnzb * (int64_t)BB, "dF");
  restrict_to(c, dF, t.it[0].mask);
  DMat dX = compact_values(c, dF, P64);
  scale_pool(c, dX.pool->vals.as<double>(), dX.pat.nnzb * (int64_t)BB, -1.0 / t.w);
  DMat X = checkpoint_copy(t, 0);
  for (int i = 1; i <= t.n_iter; ++i) {
    const TapeIter &ti = t.it[i];
    DMat nd = anticommutator(c, dX, X, ti.mask, ti.cb, ti.cc, t.step_mode(i - 1));
    dX = std::move(nd);
    if (verbose()) std::fprintf(stderr, "[sp2] jvp: step %d nnzb=%lld\n", i, (long long)dX.pat.nnzb);
    if (i < t.n_iter) X = replay_step(c, t, i, X);
  }
  return export_bsr(c, dX);
}

sp2_bsr *run_replay(Ctx &c, const Tape &t, const sp2_bsr *Fin) {
  check_same_n(t, Fin, "F");
  DMat F = borrow_matrix(c, Fin, "F");
  check_finite(c, Fin->val, Fin->nnzb * (int64_t)BB, "F");
  DMat X = init_x0(c, F, t.lmax, t.w);
  restrict_to(c, X, t.it[0].mask);
  if (t.it[0].prec == P32) X = compact_values(c, X, P32);
  for (int i = 1; i <= t.n_iter; ++i) X = replay_step(c, t, i, X);
  if (X.pool->prec == P32) {  // as the forward: a low-precision result is returned symmetrized
    X = compact_values(c, X, P32);
    sym_diag(c, X, 1.0);
  }
  return export_bsr(c, X);
}

template <typename Fn> int guarded(sp2_ctx *ctx, Fn &&fn) {
  if (!ctx) return SP2_ERR_INVALID_ARG;
  ctx->last_error.clear();
  try {
    SP2_HIP(hipSetDevice(ctx->device));
    return fn();
  } catch (const Exc &e) {
    ctx->last_error = e.msg;
    (void)hipGetLastError();
    return e.code;
  } catch (const std::bad_alloc &) {
    ctx->last_error = "host allocation failed";
    return SP2_ERR_OOM;
  } catch (const std::exception &e) {
    ctx->last_error = e.what();
    return SP2_ERR_HIP;
  }
}

}  // namespace
}  // namespace sp2

// ================================================= no-allocation scratch
// Device scratch of sp2_matrix_norms_noalloc: block norms, row indices,
// flags and partial sums live here instead of in allocated buffers.  Every
// device the library runs on holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (the array's name in host code is not a device address).
namespace sp2 {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;
}  // namespace sp2

static __device__ __align__(256) unsigned char scratch[sp2::NOALLOC_SCRATCH_BYTES];

namespace sp2 {
namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on `device`, looked up once per device with that
// device current (sp2_create has made it current)
void *scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace sp2

// ====================================================================== C ABI
using namespace sp2;

extern "C" {

const char *sp2_version(void) { return "sp2dm 0.1 gfx950"; }

void sp2_options_default(sp2_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->accel = 1;
  o->precision = SP2_PREC_FP64;
  o->switch_tol = 1e-3;
  o->trunc_norm = SP2_TRUNC_FROBINF;
  o->n_max_cap = 100;
  o->coarse_bs = 4096;
  o->gamma = 1e-3;
  o->tau_fixed = 0.0;
  o->idem_stop = 0.0;
  o->record_tape = 0;
  o->n_checkpoints = 0;
  o->correct = 0;
  o->corr_purify = 2;
  o->corr_tol = 1e-9;
  o->corr_mem = 0;
  o->adjoint_precision = -1;
}

int sp2_create(sp2_ctx **ctx, int device, void *hip_stream) {
  if (!ctx) return SP2_ERR_INVALID_ARG;
  *ctx = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SP2_ERR_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) return SP2_ERR_HIP;
  void *scr = scratch_setup(device);
  if (!scr) return SP2_ERR_HIP;
  auto *c = new sp2_ctx();
  c->device = device;
  c->scratch = scr;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *ctx = c;
  return SP2_OK;
}

void sp2_destroy(sp2_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->copy_stream) {
    (void)hipStreamSynchronize(ctx->copy_stream);
    (void)hipStreamDestroy(ctx->copy_stream);
  }
  ctx->trim();
  delete ctx;
}

int sp2_set_allocator(sp2_ctx *ctx, sp2_alloc_fn alloc, sp2_free_fn free_, void *user) {
  return guarded(ctx, [&]() {
    if ((alloc == nullptr) != (free_ == nullptr)) fail(SP2_ERR_INVALID_ARG, "give both alloc and free or neither");
    ctx->sync();
    ctx->trim();
    ctx->ualloc = alloc;
    ctx->ufree = free_;
    ctx->uuser = user;
    return SP2_OK;
  });
}

void sp2_trim(sp2_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  ctx->trim();
}

const char *sp2_last_error(const sp2_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "NULL context"; }

int sp2_gershgorin(sp2_ctx *ctx, const sp2_bsr *F, double *lmin, double *lmax) {
  return guarded(ctx, [&]() {
    if (!lmin || !lmax) fail(SP2_ERR_INVALID_ARG, "NULL output");
    DMat M = borrow_matrix(*ctx, F, "F");
    check_finite(*ctx, F->val, F->nnzb * (int64_t)BB, "F");
    Maps m = build_maps(*ctx, M.pat, true);
    Buf lo = ctx->alloc(sizeof(double) * M.pat.nbr), hi = ctx->alloc(sizeof(double) * M.pat.nbr);
    launch_gershgorin(*ctx, m.idxmap.as<int32_t>(), m.adj_ptr.as<int64_t>(), m.adj_col.as<int32_t>(),
                      M.pool->vals.as<double>(), M.pat.nbr, M.pat.n, lo.as<double>(), hi.as<double>());
    Buf out = ctx->alloc(2 * sizeof(double));
    launch_minmax(*ctx, lo.as<double>(), hi.as<double>(), M.pat.nbr, out.as<double>());
    double h[2];
    ctx->d2h(h, out.p, sizeof(h));
    *lmin = h[0];
    *lmax = h[1];
    return SP2_OK;
  });
}

int sp2_density(sp2_ctx *ctx, const sp2_bsr *F, int64_t n_occ, double lmin, double lmax, const double *homo_ub,
                const double *lumo_lb, const sp2_options *opt, sp2_bsr **D_out, double *homo_est, double *lumo_est,
                sp2_stats *stats, sp2_tape **tape) {
  return guarded(ctx, [&]() {
    sp2_options o;
    if (opt)
      o = *opt;
    else
      sp2_options_default(&o);
    return run_density(*ctx, F, n_occ, lmin, lmax, homo_ub, lumo_lb, o, D_out, homo_est, lumo_est, stats, tape);
  });
}

int sp2_density_begin(sp2_ctx *ctx, const sp2_bsr *F, int64_t n_occ, double lmin, double lmax,
                      const double *homo_ub, const double *lumo_lb, const sp2_options *opt, sp2_solver **solver) {
  return guarded(ctx, [&]() {
    if (!solver) fail(SP2_ERR_INVALID_ARG, "solver is NULL");
    *solver = nullptr;
    sp2_options o;
    if (opt)
      o = *opt;
    else
      sp2_options_default(&o);
    std::unique_ptr<sp2_solver> h(new sp2_solver());
    h->ctx = ctx;
    h->s.reset(new Solver(*ctx));
    h->s->begin(F, n_occ, lmin, lmax, homo_ub, lumo_lb, o);
    *solver = h.release();
    return SP2_OK;
  });
}

int sp2_density_step(sp2_ctx *ctx, sp2_solver *solver, sp2_step_info *info) {
  return guarded(ctx, [&]() {
    if (!solver || !solver->s) fail(SP2_ERR_INVALID_ARG, "solver is NULL");
    if (solver->ctx != ctx) fail(SP2_ERR_INVALID_ARG, "solver belongs to another context");
    solver->s->step();
    if (info) *info = solver->s->info;
    return SP2_OK;
  });
}

int sp2_density_end(sp2_ctx *ctx, sp2_solver *solver, sp2_bsr **D_out, double *homo_est, double *lumo_est,
                    sp2_stats *stats, sp2_tape **tape) {
  return guarded(ctx, [&]() {
    if (!solver || !solver->s) fail(SP2_ERR_INVALID_ARG, "solver is NULL");
    if (solver->ctx != ctx) fail(SP2_ERR_INVALID_ARG, "solver belongs to another context");
    if (!D_out) fail(SP2_ERR_INVALID_ARG, "D_out is NULL");
    *D_out = nullptr;
    if (tape) *tape = nullptr;
    Solver &s = *solver->s;
    if (stats && stats->capacity < s.o.n_max_cap + 1) fail(SP2_ERR_INVALID_ARG, "stats capacity < n_max_cap + 1");
    if (tape && !s.o.record_tape) fail(SP2_ERR_INVALID_ARG, "a tape needs record_tape = 1");
    return s.finish(D_out, homo_est, lumo_est, stats, tape);
  });
}

void sp2_solver_free(sp2_ctx *ctx, sp2_solver *solver) {
  if (!solver) return;
  if (ctx) (void)hipSetDevice(ctx->device);
  delete solver;
}

int sp2_vjp(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *W, sp2_bsr **Fbar_out) {
  return guarded(ctx, [&]() {
    if (!tape || !Fbar_out) fail(SP2_ERR_INVALID_ARG, "NULL tape or output");
    *Fbar_out = nullptr;
    *Fbar_out = run_vjp(*ctx, *tape, W);
    return SP2_OK;
  });
}

int sp2_jvp(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *dF, sp2_bsr **dD_out) {
  return guarded(ctx, [&]() {
    if (!tape || !dD_out) fail(SP2_ERR_INVALID_ARG, "NULL tape or output");
    *dD_out = nullptr;
    *dD_out = run_jvp(*ctx, *tape, dF);
    return SP2_OK;
  });
}

int sp2_replay(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *F, sp2_bsr **D_out) {
  return guarded(ctx, [&]() {
    if (!tape || !D_out) fail(SP2_ERR_INVALID_ARG, "NULL tape or output");
    *D_out = nullptr;
    *D_out = run_replay(*ctx, *tape, F);
    return SP2_OK;
  });
}

int sp2_tape_info(const sp2_tape *tape, int32_t *n_iter, int32_t *n_checkpoints, int64_t *device_bytes) {
  if (!tape) return SP2_ERR_INVALID_ARG;
  if (n_iter) *n_iter = tape->n_iter;
  if (n_checkpoints) *n_checkpoints = tape->n_ckpt;
  if (device_bytes) *device_bytes = tape->bytes;
  return SP2_OK;
}

int sp2_schedule(double lmin, double lmax, double homo_ub, double lumo_lb, int accel, double gamma, double tau_fixed,
                 int n_max_cap, int32_t *n_max, int32_t *n_min, int32_t *p, double *alpha, double *l, double *q,
                 double *xi, double *tau) {
  if (!(std::isfinite(lmin) && std::isfinite(lmax) && lmin < lmax)) return SP2_ERR_INVALID_ARG;
  if (!(lmin <= homo_ub && homo_ub < lumo_lb && lumo_lb <= lmax)) return SP2_ERR_BAD_BOUNDS;
  if (n_max_cap < 1 || n_max_cap > 1000 || !(gamma >= 0.0) || !(tau_fixed >= 0.0)) return SP2_ERR_INVALID_ARG;
  try {
    const Sched s = make_schedule(lmin, lmax, homo_ub, lumo_lb, accel != 0, gamma, tau_fixed, n_max_cap);
    if (n_max) *n_max = s.n_max;
    if (n_min) *n_min = s.n_min;
    for (int i = 0; i <= s.n_max; ++i) {
      if (p) p[i] = s.p[i];
      if (alpha) alpha[i] = s.alpha[i];
      if (l) l[i] = s.l[i];
      if (q) q[i] = s.q[i];
      if (xi) xi[i] = s.xi[i];
      if (tau) tau[i] = s.tau[i];
    }
  } catch (...) {
    return SP2_ERR_OOM;
  }
  return SP2_OK;
}

int sp2_homo_lumo(int bounds_mode, int n, const double *e, const double *trace, const int32_t *p, const double *alpha,
                  const double *l, const double *q, double lmin, double lmax, int64_t N, int64_t n_occ,
                  double *homo_ub, double *lumo_lb) {
  if (n < 0 || !e || !p || !alpha || !homo_ub || !lumo_lb || !(lmin < lmax)) return SP2_ERR_INVALID_ARG;
  if (bounds_mode ? (!l || !q) : !trace) return SP2_ERR_INVALID_ARG;
  try {
    Sched s;
    s.bounds = bounds_mode != 0;
    if (s.bounds) {
      s.l.assign(l, l + n + 1);
      s.q.assign(q, q + n + 1);
    }
    std::vector<double> ev(e, e + n + 1), tv(n + 1, 0.0), av(alpha, alpha + n + 1);
    if (trace) tv.assign(trace, trace + n + 1);
    std::vector<int> pv(p, p + n + 1);
    homo_lumo(s, ev, tv, pv, av, n, lmin, lmax, N, n_occ, *homo_ub, *lumo_lb);
  } catch (...) {
    return SP2_ERR_OOM;
  }
  return SP2_OK;
}

int sp2_square_step(sp2_ctx *ctx, const sp2_bsr *Xin, double a, double b, double cc, int precision,
                    sp2_bsr **Xn_out, double sums[4]) {
  return guarded(ctx, [&]() {
    if (!Xn_out) fail(SP2_ERR_INVALID_ARG, "NULL output");
    *Xn_out = nullptr;
    if (precision < 0 || precision > 2) fail(SP2_ERR_INVALID_ARG, "unknown precision");
    DMat X = borrow_matrix(*ctx, Xin, "X");
    check_finite(*ctx, Xin->val, Xin->nnzb * (int64_t)BB, "X");
    int mode = M_F64;
    if (precision != SP2_PREC_FP64) {
      X = compact_values(*ctx, X, P32);
      mode = precision == SP2_PREC_FP32 ? M_F32 : M_BF16X3;
    }
    Maps m = build_maps(*ctx, X.pat, true);
    SquareOut so = square_step(*ctx, X, m, mode, X.pool->prec, a, b, cc);
    if (sums) {
      sums[0] = so.sums[0];
      sums[1] = so.sums[1];
      sums[2] = so.sums[2];
      sums[3] = so.sums[4] * 2.0 * B * B * B;
    }
    *Xn_out = export_bsr(*ctx, so.next);
    return SP2_OK;
  });
}

int sp2_pair_product(sp2_ctx *ctx, const sp2_bsr *Xin, const sp2_bsr *Yin, const sp2_bsr *Gin, int sign, int y_antisym,
                     double a, double b, double cc, int precision, sp2_bsr **out, double sums[2]) {
  return guarded(ctx, [&]() {
    if (!out) fail(SP2_ERR_INVALID_ARG, "NULL output");
    *out = nullptr;
    if (precision < 0 || precision > 2) fail(SP2_ERR_INVALID_ARG, "unknown precision");
    if (sign != 1 && sign != -1) fail(SP2_ERR_INVALID_ARG, "sign must be +1 or -1");
    if (y_antisym != 0 && y_antisym != 1) fail(SP2_ERR_INVALID_ARG, "y_antisym must be 0 or 1");
    DMat X = borrow_matrix(*ctx, Xin, "X");
    DMat Y = borrow_matrix(*ctx, Yin, "Y");
    if (Xin->n != Yin->n) fail(SP2_ERR_INVALID_ARG, "X and Y differ in size");
    check_finite(*ctx, Xin->val, Xin->nnzb * (int64_t)BB, "X");
    check_finite(*ctx, Yin->val, Yin->nnzb * (int64_t)BB, "Y");
    DMat G;
    if (Gin) {
      G = borrow_matrix(*ctx, Gin, "G");
      if (Gin->n != Xin->n) fail(SP2_ERR_INVALID_ARG, "G differs in size");
      check_finite(*ctx, Gin->val, Gin->nnzb * (int64_t)BB, "G");
    }
    int mode = M_F64;
    if (precision != SP2_PREC_FP64) {
      X = compact_values(*ctx, X, P32);
      Y = compact_values(*ctx, Y, P32);
      if (Gin) G = compact_values(*ctx, G, P32);
      mode = precision == SP2_PREC_FP32 ? M_F32 : M_BF16X3;
    }
    Maps mx = build_maps(*ctx, X.pat, true), my = build_maps(*ctx, Y.pat, true);
    Maps mg;
    if (Gin) mg = build_maps(*ctx, G.pat, false);
    PairOpt po;
    po.neg2 = sign < 0;
    po.yanti = y_antisym != 0;
    po.G = Gin ? &G : nullptr;
    po.mg = Gin ? &mg : nullptr;
    po.ca = a;
    po.cb = b;
    po.cc = cc;
    po.mode = mode;
    po.oprec = X.pool->prec;
    SquareOut so = pair_product(*ctx, X, mx, Y, my, po);
    if (sums) {
      sums[0] = frob_norm(*ctx, so.next);
      sums[0] *= sums[0];
      sums[1] = so.sums[4] * 2.0 * B * B * B;
    }
    *out = export_bsr(*ctx, so.next);
    return SP2_OK;
  });
}

int sp2_general_from_upper(sp2_ctx *ctx, const sp2_bsr *Uin, sp2_bsr **G_out) {
  return guarded(ctx, [&]() {
    if (!G_out) fail(SP2_ERR_INVALID_ARG, "NULL output");
    *G_out = nullptr;
    DMat U = borrow_matrix(*ctx, Uin, "U");
    check_finite(*ctx, Uin->val, Uin->nnzb * (int64_t)BB, "U");
    *G_out = export_bsr(*ctx, expand_upper(*ctx, U));
    return SP2_OK;
  });
}

int sp2_general_product(sp2_ctx *ctx, const sp2_bsr *Ain, const sp2_bsr *Bin, const sp2_bsr *Gin, double a, double b,
                        double cc, int precision, sp2_bsr **out, double sums[4]) {
  return guarded(ctx, [&]() {
    if (!out) fail(SP2_ERR_INVALID_ARG, "NULL output");
    *out = nullptr;
    if (precision != SP2_PREC_FP64 && precision != SP2_PREC_BF16X3)
      fail(SP2_ERR_INVALID_ARG, "general product: precision must be SP2_PREC_FP64 or SP2_PREC_BF16X3");
    DMat A = borrow_matrix(*ctx, Ain, "A", true);
    DMat Bm = borrow_matrix(*ctx, Bin, "B", true);
    if (Ain->n != Bin->n) fail(SP2_ERR_INVALID_ARG, "A and B differ in size");
    check_finite(*ctx, Ain->val, Ain->nnzb * (int64_t)BB, "A");
    check_finite(*ctx, Bin->val, Bin->nnzb * (int64_t)BB, "B");
    DMat G;
    if (Gin) {
      G = borrow_matrix(*ctx, Gin, "G", true);
      if (Gin->n != Ain->n) fail(SP2_ERR_INVALID_ARG, "G differs in size");
      check_finite(*ctx, Gin->val, Gin->nnzb * (int64_t)BB, "G");
    }
    const int mode = precision == SP2_PREC_FP64 ? M_F64 : M_BF16X3;
    if (mode != M_F64) {
      A = compact_values(*ctx, A, P32);
      Bm = compact_values(*ctx, Bm, P32);
      if (Gin) G = compact_values(*ctx, G, P32);
    }
    SquareOut so = general_product(*ctx, A, Bm, Gin ? &G : nullptr, a, b, cc, mode);
    if (sums) {
      sums[0] = so.sums[0];
      sums[1] = so.sums[1];
      sums[2] = so.sums[2];
      sums[3] = so.sums[4] * 2.0 * B * B * B;
    }
    *out = export_bsr(*ctx, so.next);
    return SP2_OK;
  });
}

int sp2_truncate(sp2_ctx *ctx, const sp2_bsr *Xin, double tau, int norm, int64_t coarse_bs, sp2_bsr **Xt_out,
                 double err[2]) {
  return guarded(ctx, [&]() {
    if (!Xt_out) fail(SP2_ERR_INVALID_ARG, "NULL output");
    *Xt_out = nullptr;
    if (norm < 0 || norm > 2) fail(SP2_ERR_INVALID_ARG, "unknown truncation norm");
    if (!(tau >= 0.0)) fail(SP2_ERR_INVALID_ARG, "tau must be >= 0");
    DMat X = borrow_matrix(*ctx, Xin, "X");
    check_finite(*ctx, Xin->val, Xin->nnzb * (int64_t)BB, "X");
    // diagonal blocks are never removed: the input must store all of them
    {
      Buf cnt = ctx->alloc(sizeof(int64_t) * X.pat.nbr);
      launch_diag_missing(*ctx, X.pat.row_ptr.as<int64_t>(), X.pat.col_idx.as<int32_t>(), X.pat.nbr,
                          cnt.as<int64_t>());
      Buf tot = ctx->alloc(sizeof(int64_t) * (X.pat.nbr + 1));
      scan_exclusive_i64(*ctx, cnt.as<int64_t>(), tot.as<int64_t>(), X.pat.nbr);
      int64_t t = 0;
      ctx->d2h(&t, tot.as<int64_t>() + X.pat.nbr, sizeof(t));
      if (t != X.pat.nnzb) fail(SP2_ERR_INVALID_ARG, "X must store every diagonal block");
    }
    Buf nrm2 = norms_of(*ctx, X);
    TruncResult tr = truncate_matrix(*ctx, X, nrm2.as<double>(), tau, norm, coarse_bs);
    if (err) {
      err[0] = tr.err_frob;
      err[1] = tr.err_mixed;
    }
    *Xt_out = export_bsr(*ctx, X);
    return SP2_OK;
  });
}

int sp2_matrix_norms(sp2_ctx *ctx, const sp2_bsr *Ain, int64_t coarse_bs, double *frob, double *frobinf) {
  return guarded(ctx, [&]() {
    if (frobinf && (coarse_bs <= 0 || coarse_bs % B))
      fail(SP2_ERR_INVALID_ARG, "coarse_bs must be a positive multiple of 64");
    DMat A = borrow_matrix(*ctx, Ain, "A");
    check_finite(*ctx, Ain->val, Ain->nnzb * (int64_t)BB, "A");
    if (frob) *frob = frob_norm(*ctx, A);
    if (frobinf) {
      *frobinf = 0.0;
      const int nbr = (int)A.pat.nbr, cb = (int)(coarse_bs / B);
      const int nc = (nbr + cb - 1) / cb;
      if (nc > 16384) fail(SP2_ERR_INVALID_ARG, "coarse_bs too small for this matrix (more than 16384 submatrices per row)");
      if (A.pat.nnzb > 0 && nc > 0) {
        Buf nrm2 = norms_of(*ctx, A);
        Buf pair = ctx->alloc(sizeof(double) * ((size_t)nc * (nc + 1) / 2));
        Buf rows = ctx->alloc(sizeof(double) * nc);
        launch_coarse_rowsums(*ctx, A.pat.row_ptr.as<int64_t>(), A.pat.col_idx.as<int32_t>(), nrm2.as<double>(), nbr,
                              cb, nc, pair.as<double>(), rows.as<double>());
        std::vector<double> h(nc);
        ctx->d2h(h.data(), rows.p, sizeof(double) * nc);
        for (double v : h) *frobinf = std::max(*frobinf, v);
      }
    }
    return SP2_OK;
  });
}

int sp2_matrix_norms_noalloc(sp2_ctx *ctx, const sp2_bsr *Ain, int64_t coarse_bs, double *frob, double *frobinf) {
  return guarded(ctx, [&]() {
    Ctx &c = *ctx;
    if (!c.scratch) fail(SP2_ERR_HIP, "device scratch of the no-allocation entry point is not set up");
    if (frobinf && (coarse_bs <= 0 || coarse_bs % B))
      fail(SP2_ERR_INVALID_ARG, "coarse_bs must be a positive multiple of 64");
    check_input(Ain, "A");
    const int64_t nnzb = Ain->nnzb;
    const int nbr = (int)Ain->nbr, cb = frobinf ? (int)(coarse_bs / B) : 1;
    const int nc = frobinf ? (nbr + cb - 1) / cb : 0;
    if (nc > 16384) fail(SP2_ERR_INVALID_ARG, "coarse_bs too small for this matrix (more than 16384 submatrices per row)");
    const int64_t npairs = (int64_t)nc * (nc + 1) / 2;
    // scratch layout: row of each block, block norms, flag, sum, reduction
    // stage, coarse pair sums, coarse row sums
    const size_t nb = (size_t)std::max<int64_t>(nnzb, 1);
    size_t off = 0;
    const size_t o_row = off;
    off += align256(sizeof(int32_t) * nb);
    const size_t o_nrm = off;
    off += align256(sizeof(double) * nb);
    const size_t o_flag = off;
    off += 256;
    const size_t o_sum = off;
    off += 256;
    const size_t o_stage = off;
    off += align256(sizeof(double) * (size_t)reduce_stage_doubles(1));
    const size_t o_pair = off;
    off += align256(sizeof(double) * (size_t)std::max<int64_t>(npairs, 1));
    const size_t o_rows = off;
    off += align256(sizeof(double) * (size_t)std::max(nc, 1));
    if (off > NOALLOC_SCRATCH_BYTES)
      fail(SP2_ERR_INVALID_ARG, "matrix too large for sp2_matrix_norms_noalloc: needs " + std::to_string(off) +
                                    " bytes of device scratch, the maximum is " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + " (about 5.5 million stored blocks)");
    char *sc = static_cast<char *>(c.scratch);
    int32_t *row_of = reinterpret_cast<int32_t *>(sc + o_row);
    double *nrm2 = reinterpret_cast<double *>(sc + o_nrm);
    int32_t *flag = reinterpret_cast<int32_t *>(sc + o_flag);
    double *sum = reinterpret_cast<double *>(sc + o_sum);
    double *stage = reinterpret_cast<double *>(sc + o_stage);
    double *pair = reinterpret_cast<double *>(sc + o_pair);
    double *rows = reinterpret_cast<double *>(sc + o_rows);
    // the pattern and value checks of sp2_matrix_norms
    std::vector<int64_t> rp(nbr + 1);
    c.d2h(rp.data(), Ain->row_ptr, sizeof(int64_t) * (nbr + 1));
    if (rp[0] != 0 || rp[nbr] != nnzb) fail(SP2_ERR_INVALID_ARG, "A: row_ptr ends");
    for (int r = 0; r < nbr; ++r)
      if (rp[r + 1] < rp[r]) fail(SP2_ERR_INVALID_ARG, "A: row_ptr not monotone");
    int32_t f = 0;
    launch_row_of(c, Ain->row_ptr, nbr, row_of);
    launch_fill_i32(c, flag, 1, 0);
    launch_validate_pattern(c, Ain->row_ptr, Ain->col_idx, nbr, nnzb, flag);
    c.d2h(&f, flag, sizeof(f));
    if (f) fail(SP2_ERR_INVALID_ARG, "A: columns must satisfy row <= col < nbr, strictly increasing");
    launch_fill_i32(c, flag, 1, 0);
    launch_check_finite(c, Ain->val, nnzb * (int64_t)BB, flag);
    c.d2h(&f, flag, sizeof(f));
    if (f) fail(SP2_ERR_NONFINITE, "A holds non-finite values");
    if (frob) {
      *frob = 0.0;
      if (nnzb > 0) {
        launch_block_norms(c, Ain->val, P64, nullptr, nnzb, nrm2);
        launch_weight_offdiag(c, nrm2, row_of, Ain->col_idx, nnzb);
        launch_reduce_parts(c, nrm2, nnzb, 1, sum, stage);
        double v = 0.0;
        c.d2h(&v, sum, sizeof(double));
        *frob = std::sqrt(std::fmax(v, 0.0));
      }
    }
    if (frobinf) {
      *frobinf = 0.0;
      if (nnzb > 0 && nc > 0) {
        launch_block_norms(c, Ain->val, P64, nullptr, nnzb, nrm2);
        launch_coarse_rowsums(c, Ain->row_ptr, Ain->col_idx, nrm2, nbr, cb, nc, pair, rows);
        std::vector<double> h(nc);
        c.d2h(h.data(), rows, sizeof(double) * nc);
        for (double v : h) *frobinf = std::max(*frobinf, v);
      }
    }
    return SP2_OK;
  });
}

int sp2_bsr_copy(sp2_ctx *ctx, const sp2_bsr *src, int64_t *row_ptr, int32_t *col_idx, double *val) {
  return guarded(ctx, [&]() {
    if (!src) fail(SP2_ERR_INVALID_ARG, "NULL matrix");
    if (!row_ptr || (src->nnzb > 0 && (!col_idx || !val))) fail(SP2_ERR_INVALID_ARG, "NULL destination");
    SP2_HIP(hipMemcpyAsync(row_ptr, src->row_ptr, sizeof(int64_t) * (src->nbr + 1), hipMemcpyDeviceToDevice,
                           ctx->stream));
    if (src->nnzb > 0) {
      SP2_HIP(hipMemcpyAsync(col_idx, src->col_idx, sizeof(int32_t) * src->nnzb, hipMemcpyDeviceToDevice,
                             ctx->stream));
      SP2_HIP(hipMemcpyAsync(val, src->val, sizeof(double) * BB * src->nnzb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    ctx->sync();
    return SP2_OK;
  });
}

void sp2_bsr_free(sp2_ctx *ctx, sp2_bsr *m) {
  if (!m || !m->owned) return;
  if (ctx) (void)hipSetDevice(ctx->device);
  delete reinterpret_cast<OwnedBsr *>(m);
}

void sp2_tape_free(sp2_ctx *ctx, sp2_tape *tape) {
  if (!tape) return;
  if (ctx) (void)hipSetDevice(ctx->device);
  delete tape;
}

}  // extern "C"
