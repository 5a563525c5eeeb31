// Internal declarations of the SP2 density-matrix library (gfx950).
//
// Device data layout
// ------------------
// A symmetric block-sparse matrix is held as
//   * a pattern: upper-triangle block rows (row_ptr int64[nbr+1], col_idx
//     int32[nnzb] sorted, row_of int32[nnzb]) plus slot int32[nnzb], the
//     position of each block in a value pool;
//   * a value pool: nslots blocks of 64 x 64 row-major values, double or
//     float.  Truncation only rewrites the pattern: surviving blocks keep their
//     slot, so values are never copied between iterations.
// Derived per pattern (Maps):
//   * idxmap int32[nbr * nbr]: slot of block (min(I,K), max(I,K)) or -1, so
//     both X_IK and its transpose are found in O(1);
//   * bits uint32[nbr * W], W = ceil(nbr / 32): row I has bit K set when X_IK
//     is stored (either orientation);
//   * adjacency (adj_ptr, adj_col): the set bits of every row, in order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "sp2dm.h"

namespace sp2 {

constexpr int B = 64;          // block size
constexpr int BB = B * B;      // elements per block
constexpr int MAX_NBR = 32768; // dense block maps are nbr^2 int32
constexpr size_t BIG_BUFFER = (size_t)64 << 20;  // device buffers above this size are rounded coarsely
constexpr size_t FREE_RESERVE = (size_t)8 << 30;  // device memory kept free of cached library buffers

struct Exc {
  int code;
  std::string msg;
};
[[noreturn]] inline void fail(int code, const std::string &msg) { throw Exc{code, msg}; }

#define SP2_HIP(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      ::sp2::fail(e_ == hipErrorOutOfMemory ? SP2_ERR_OOM : SP2_ERR_HIP,                \
                  std::string(#x) + ": " + hipGetErrorString(e_));                      \
  } while (0)

#define SP2_LAUNCH_CHECK() SP2_HIP(hipGetLastError())

enum Prec : int { P64 = 0, P32 = 1 };  // storage precision of a value pool
enum Mode : int { M_F64 = 0, M_F32 = 1, M_BF16X3 = 2 };  // arithmetic of a square

struct Ctx;

// ---------------------------------------------------------------- buffers
struct Buf {
  Ctx *ctx = nullptr;
  void *p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  Buf(Buf &&o) noexcept { *this = std::move(o); }
  Buf &operator=(Buf &&o) noexcept;
  ~Buf() { reset(); }
  void reset();
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  sp2_alloc_fn ualloc = nullptr;
  sp2_free_fn ufree = nullptr;
  void *uuser = nullptr;
  std::string last_error;
  std::multimap<size_t, void *> cache;  // released buffers, reused by size
  size_t cached_bytes = 0;
  size_t live_bytes = 0, peak_bytes = 0;
  // device time (HIP events) and algorithmic flops of the MFMA product kernels
  // launched so far, by arithmetic (Mode); read by the stepped solver
  double kern_s[3] = {0.0, 0.0, 0.0};
  double kern_flops[3] = {0.0, 0.0, 0.0};
  int64_t kern_launches[3] = {0, 0, 0};
  // calls into the device allocator and the host time they took
  int64_t n_raw_alloc = 0, n_raw_free = 0;
  double raw_alloc_s = 0.0, raw_free_s = 0.0;
  double *h_pinned = nullptr;  // pinned host staging for small device->host reads
  size_t h_pinned_bytes = 0;

  // device address of the no-allocation entry point's scratch array on this
  // context's device (set by sp2_create)
  void *scratch = nullptr;
  // second stream (default priority) for host <-> device copies that overlap
  // the kernels of `stream`; created on first use
  hipStream_t copy_stream = nullptr;
  hipStream_t copies();

  Buf alloc(size_t bytes);
  void release(void *p, size_t bytes);
  void trim();
  void sync();
  // small device -> host copy through pinned staging, then stream sync
  void d2h(void *dst, const void *src, size_t bytes);
  void h2d(void *dst, const void *src, size_t bytes);
  void *raw_alloc(size_t bytes);
  void raw_free(void *p);
};

// ---------------------------------------------------------------- matrices
struct Pattern {
  int64_t n = 0;
  int nbr = 0;
  int64_t nnzb = 0;
  Buf row_ptr;  // int64[nbr+1]
  Buf col_idx;  // int32[nnzb]
  Buf row_of;   // int32[nnzb]
  Buf slot;     // int32[nnzb]
};

struct Maps {
  int nbr = 0, W = 0;
  Buf idxmap;   // int32[nbr*nbr]
  Buf bits;     // uint32[nbr*W]
  Buf adj_ptr;  // int64[nbr+1]
  Buf adj_col;  // int32[adj_ptr[nbr]]
  int64_t nadj = 0;
};

struct Pool {
  Buf vals;
  int prec = P64;
  int64_t nslots = 0;
  std::shared_ptr<Buf> keep;  // shared ownership when a tape also holds it
};

struct DMat {
  Pattern pat;
  std::shared_ptr<Pool> pool;
};

// ---------------------------------------------------------------- launchers
// pattern / maps (kernels_pattern.hip)
void launch_fill_i32(Ctx &c, int32_t *p, int64_t n, int32_t v);
void launch_fill_u32(Ctx &c, uint32_t *p, int64_t n, uint32_t v);
void launch_fill_f64(Ctx &c, double *p, int64_t n, double v);
void launch_iota_i32(Ctx &c, int32_t *p, int64_t n);
void launch_row_of(Ctx &c, const int64_t *row_ptr, int nbr, int32_t *row_of);
void launch_validate_pattern(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb,
                             int32_t *flag);
void launch_build_maps(Ctx &c, const int32_t *row_of, const int32_t *col_idx, const int32_t *slot, int64_t nnzb,
                       int nbr, int W, int32_t *idxmap, uint32_t *bits);
void launch_popcount_rows(Ctx &c, const uint32_t *bits, int nbr, int W, int64_t *counts);
void launch_extract_rows(Ctx &c, const uint32_t *bits, int nbr, int W, const int64_t *ptr, int32_t *cols,
                         int32_t *rows);
// outbits row I (J >= I only) = OR of bits[K] over K in adj row I; with a
// second (bits2, adj2) set also OR of bits2[K] over K in adj2 row I
// (upper = false: every column J, for general storage)
void launch_symbolic(Ctx &c, const uint32_t *bits, const int64_t *adj_ptr, const int32_t *adj_col, int nbr, int W,
                     uint32_t *outbits, const uint32_t *bits2 = nullptr, const int64_t *adj_ptr2 = nullptr,
                     const int32_t *adj_col2 = nullptr, bool upper = true);
// general storage (kernels_general.hip): flag |= 1 for a column outside [0, nbr),
// 2 for columns not strictly increasing, 4 for a non-monotone row_ptr
void launch_validate_general(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t nnzb,
                             int32_t *flag);
// block map and bitmaps of a general pattern: idxmap[R nbr + C] = slot and bit C
// of bits row R, with (R, C) = (I, J), or (J, I) for transpose; idxmap may be null
void launch_build_maps_general(Ctx &c, const int32_t *row_of, const int32_t *col_idx, const int32_t *slot,
                               int64_t nnzb, int nbr, int W, bool transpose, int32_t *idxmap, uint32_t *bits);
// out |= g (if not null), and the diagonal bits with diag
void launch_or_general(Ctx &c, uint32_t *out, const uint32_t *g, int nbr, int W, bool diag);
// general storage of a symmetric upper-BSR matrix: output block (I, J) (pattern
// row_of / col) is the stored block idxmap[I nbr + J] of src, transposed for I > J
void launch_expand_upper(Ctx &c, const int32_t *row_of, const int32_t *col, int64_t nout, int nbr,
                         const int32_t *idxmap, const double *src, double *dst);
// out = upper part (J >= I) of a | b (symmetric block-row bitmaps)
void launch_or_upper(Ctx &c, const uint32_t *a, const uint32_t *b, int nbr, int W, uint32_t *out);
// out (FP64, by output position) = a A + b B over an output pattern given by (row_of, col)
void launch_add_union(Ctx &c, const int32_t *row_of, const int32_t *col, int64_t nblocks, int nbr, const void *pa,
                      int preca, const int32_t *ia, double a, const void *pb, int precb, const int32_t *ib, double b,
                      double *out);
// diagonal blocks (B + sign B^T) / 2 in place (sign = 1 symmetric, -1 antisymmetric)
void launch_sym_diag(Ctx &c, void *pool, int prec, const int64_t *row_ptr, const int32_t *col_idx,
                     const int32_t *slot, int nbr, double sign);
// nrm2[b] *= 2 for off-diagonal blocks (whole-matrix Frobenius weights)
void launch_weight_offdiag(Ctx &c, double *nrm2, const int32_t *row_of, const int32_t *col, int64_t nblocks);
// exclusive scan of n int64 counts into out[0..n] (out[n] = total)
void scan_exclusive_i64(Ctx &c, const int64_t *in, int64_t *out, int64_t n);
void launch_diag_missing(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, int nbr, int64_t *counts);
void launch_x0_pattern(Ctx &c, const int64_t *frow_ptr, const int32_t *fcol, int nbr, const int64_t *xrow_ptr,
                       int32_t *xcol, int32_t *src);
void launch_init_x0(Ctx &c, const double *fval, const int32_t *src, const int32_t *xrow_of, const int32_t *xcol,
                    int64_t nnzb, int64_t n, double lmax, double w, double *xval);

// values (kernels_values.hip)
void launch_check_finite(Ctx &c, const double *v, int64_t n, int32_t *flag);
void launch_gershgorin(Ctx &c, const int32_t *idxmap, const int64_t *adj_ptr, const int32_t *adj_col,
                       const double *val, int nbr, int64_t n, double *row_lo, double *row_hi);
void launch_minmax(Ctx &c, const double *lo, const double *hi, int n, double *out2);
void launch_gather(Ctx &c, const void *src, int src_prec, const int32_t *slot, int64_t nblocks, void *dst,
                   int dst_prec);
void launch_reduce_parts(Ctx &c, const double *parts, int64_t nrows, int ncols, double *out);
// the same reduction with a caller-supplied staging buffer of reduce_stage_doubles(ncols) doubles
void launch_reduce_parts(Ctx &c, const double *parts, int64_t nrows, int ncols, double *out, double *stage);
constexpr int64_t reduce_stage_doubles(int ncols) { return (int64_t)256 * ncols; }
void launch_block_norms(Ctx &c, const void *pool, int prec, const int32_t *slot, int64_t nblocks, double *nrm2);
// pair: nc (nc + 1) / 2 doubles (packed upper coarse squared norms); rowsum: nc
void launch_coarse_rowsums(Ctx &c, const int64_t *row_ptr, const int32_t *col_idx, const double *nrm2, int nbr,
                           int cb, int nc, double *pair, double *rowsum);
void launch_update(Ctx &c, const void *xpool, int xprec, const int32_t *xidxmap, int nbr, const int32_t *out_row,
                   const int32_t *out_col, int64_t nout, void *spool, int sprec, double ca, double cb, double cc,
                   int64_t n, double *parts);

constexpr int NPART = 5;  // per output block: e2 (weighted), trX, trS, ||out||^2, #K

// tiled square: one workgroup per 2 x 2 tile of output blocks (kernels_tile.hip)
// Tiled block product with symmetric (or antisymmetric) upper-stored operands
// and an output on a given upper pattern:
//   acc(I, J) = sum_K X_IK Y_KJ  [+ s2 * sum_K Y_IK X_KJ when npass == 2]
//   out(I, J) = ca [I == J] I + cb G_IJ + cc acc(I, J)
// The square of Algorithm 2 is X == Y, npass == 1, G == X.  A lower block of
// an antisymmetric source (xanti / yanti) is minus the transpose of the stored
// upper block.
struct TileArgs {
  const void *xpool;
  int xprec;
  const int32_t *idxmap;   // slot map of X (symmetric: (I, J) and (J, I) give the stored block)
  const uint32_t *bits;    // block-row bitmaps of X
  const void *ypool;       // second operand Y (same precision as X)
  const int32_t *yidxmap;
  const uint32_t *ybits;
  int npass = 1;           // 1: X Y; 2: X Y + s2 Y X
  int neg2 = 0;            // s2 = -1
  int xanti = 0, yanti = 0;
  const void *xpack = nullptr, *ypack = nullptr;  // BF16x3: operands split into bf16 images (launch_pack_bf16x3)
  const void *gpool;       // G of the cb term (same precision as X), or null
  const int32_t *gidxmap;
  int nbr, W;
  const int32_t *oidx;     // nbr x nbr: pattern position of output block (I, J), or -1
  const int32_t *tiles;    // ntiles pairs (TI, TJ), TI <= TJ in units of tb blocks
  int tb = 2;              // tile edge in blocks: 2 (every kernel) or 4 (BF16x3, dense patterns)
  int full = 0;            // general storage: X (direct map, row bitmaps) times Y (map and bitmaps of Y^T),
                           // every block stored as is (no transposed reads), output tiles of both triangles
  int64_t ntiles;
  int64_t xcd_chunk;       // tiles per XCD: workgroup b runs tile (b % 8) * xcd_chunk + b / 8
  void *opool;             // output block at its pattern position
  int oprec;
  double ca, cb, cc;
  int64_t n;
  double *parts;           // by pattern position, NPART each
};
// output tiles holding at least one output block: TI <= TJ (upper output), or
// every tile with full = true (general storage)
int64_t build_tiles(Ctx &c, const int32_t *oidx, int nbr, Buf &tiles, int tb = 2, bool full = false);
void launch_square_tile(Ctx &c, int mode, const TileArgs &a);
// FP64 squares and products with operands loaded straight to LDS (kernels_f64.hip)
// (FP64 operands, or FP32-stored ones widened to FP64 at the fragment reads)
void launch_square_f64_lds(Ctx &c, const TileArgs &a);
void launch_square_tile_bf16x3(Ctx &c, const TileArgs &a);  // kernels_bf16x3.hip
// split the stored blocks of an FP32 pool into bf16 hi/lo images of the block
// and of its transpose: packed[slot] = 4 x 4096 bf16 (32 KB per pool slot)
void launch_pack_bf16x3(Ctx &c, const float *pool, const int32_t *slot, int64_t nblocks, uint16_t *packed);

// truncation (kernels_trunc.hip)
struct TruncOut {
  std::vector<double> seg_err;  // per segment removed weighted sum
  int64_t removed = 0;
};
// keep[b] (int64, 1 = kept) for every stored block; per-segment removed sums
void truncate_select(Ctx &c, const Pattern &pat, const double *nrm2_by_block, double tau, int norm,
                     int64_t coarse_bs, int64_t *keep, TruncOut &out, int nc_out[1]);
void compact_pattern(Ctx &c, const Pattern &in, const int64_t *keep, Pattern &out);
void launch_mark_in_mask(Ctx &c, const Pattern &pat, const uint32_t *mask_bits, int W, int64_t *keep);

}  // namespace sp2
