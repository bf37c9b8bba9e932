// internal.h -- shared host-side declarations of libbsmm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "bsmm.h"

namespace bsmm {

// Thrown inside the library, converted to a status at the ABI boundary.
struct Error {
  bsmm_status code;
  std::string msg;
};

[[noreturn]] void fail(bsmm_status code, const std::string &msg);
// Detail returned by bsmm_last_error() on this host thread.
void set_last_error(const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPCHECK(x) ::bsmm::hip_check((x), #x, __FILE__, __LINE__)

// Caching device allocator.  All work of one context is ordered on one
// stream, so a buffer freed here can be handed out again at once: any later
// use is queued behind the work that used it before.
class Allocator {
 public:
  void init(int device, size_t budget);
  void *alloc(size_t bytes);
  void release(void *p);
  void trim();             // return cached free blocks to HIP
  size_t held() const { return held_; }
  size_t peak() const { return peak_; }
  // Fails with BSMM_ERR_OUT_OF_MEMORY when `bytes` more in live buffers
  // would exceed the budget (cached free blocks count as available).
  void check(size_t bytes, const char *what) const;
  // Bytes that live buffers may still grow by under the budget (SIZE_MAX
  // without one).
  size_t room() const;
  ~Allocator();

 private:
  int device_ = 0;
  size_t budget_ = 0;      // 0 = no cap
  size_t held_ = 0, peak_ = 0;
  size_t cached_ = 0;      // bytes of the free blocks in the cache
  std::multimap<size_t, void *> free_;   // size -> ptr
  std::map<void *, size_t> live_;        // ptr -> size
};

}  // namespace bsmm

// Body of every ABI entry point: library errors become status codes.
#define ABI_BEGIN try {
#define ABI_END                                              \
  return BSMM_OK;                                            \
  }                                                          \
  catch (const ::bsmm::Error &e) {                           \
    ::bsmm::set_last_error(e.msg);                           \
    return e.code;                                           \
  }                                                          \
  catch (const std::bad_alloc &) {                           \
    ::bsmm::set_last_error("host allocation failed");        \
    return BSMM_ERR_OUT_OF_MEMORY;                           \
  }                                                          \
  catch (...) {                                              \
    ::bsmm::set_last_error("unexpected internal error");     \
    return BSMM_ERR_DEVICE;                                  \
  }

struct bsmm_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool timing = false;
  bsmm_compute_mode mode = BSMM_COMPUTE_FP64;
  bsmm::Allocator alloc;
  int64_t *pinned = nullptr;   // small host buffer for size read-backs
  uint8_t gemm_variant[16] = {};   // GEMM kernel variant per (m, n) size class
  int tile_ti = 2, tile_tj = 2;    // result-block tile of the tile path
  int64_t tile_chunk = 0;          // tiles per XCD chunk of the tile path (0: 8192)
  int32_t pack_addr = 0;           // packed-operand addressing: 0 = automatic, 1 = per row / column
  int32_t row_order = 0;           // locality order of square operands: 0 = automatic, 1 = always, 2 = never
  // Staging of batched launch parameters: a ring of pinned host slots, each
  // reused once the copy from it has run (its event), and one device buffer
  // (every copy into it is ordered after the previous launch on the stream).
  static constexpr int NSTAGE = 4;
  void *stage_host[NSTAGE] = {};
  hipEvent_t stage_ev[NSTAGE] = {};
  int stage_next = 0;
  void *batch_dev = nullptr;
  size_t batch_bytes = 0;
  double *zeros = nullptr;     // 4 KB zero page on the device
  int live_mats = 0;
};

struct bsmm_mat_s {
  bsmm_ctx ctx = nullptr;
  int32_t nbr = 0, nbc = 0;
  int64_t nnzb = 0, n_values = 0;
  std::vector<int32_t> h_rbs, h_cbs;   // block sizes (host copy)
  int32_t *d_rbs = nullptr, *d_cbs = nullptr;
  int64_t *d_row_ptr = nullptr;        // nbr+1
  int32_t *d_col_idx = nullptr;        // nnzb
  int64_t *d_blk_off = nullptr;        // nnzb+1 element offsets (the prefix of the block areas)
  double *d_values = nullptr;
  bool owns_values = false;
  // planner cache: locality order of the block rows (host and device copy)
  std::vector<int32_t> h_order;
  int32_t *d_order = nullptr;
};

namespace bsmm {

// RAII device buffer from the context allocator.
template <typename T>
struct DBuf {
  Allocator *a = nullptr;
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(Allocator &al, size_t count) : a(&al), p(nullptr), n(count) {
    if (count) p = static_cast<T *>(al.alloc(count * sizeof(T)));
  }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : a(o.a), p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) { reset(); a = o.a; p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() { if (p && a) a->release(p); p = nullptr; n = 0; }
  T *release_ownership() { T *q = p; p = nullptr; n = 0; return q; }
};

// ----------------------------------------------------------- kernel launchers
// Each launcher enqueues on `s`; sizes are validated by the caller.

// out[i] = sum_{t<i} in[t] for i = 0..n (out has n+1 entries); the total
// ends in out[n].  `tmp` comes from the allocator.
void exclusive_scan_i64(Allocator &al, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
void exclusive_scan_i32(Allocator &al, const int32_t *in, int64_t *out, int64_t n, hipStream_t s);

// Operand view: rows of op(X) with the original block id of every entry.
struct OpIndex {
  int32_t nbr = 0, nbc = 0;          // block grid of op(X)
  const int64_t *row_ptr = nullptr;  // nbr+1
  const int32_t *col_idx = nullptr;  // entries, sorted per row
  const int32_t *blk = nullptr;      // original block id per entry (nullptr = identity)
  const int32_t *rbs = nullptr, *cbs = nullptr;   // block sizes of op(X) (device)
  const int64_t *blk_off = nullptr;  // value offsets of the original blocks
  const double *values = nullptr;
  bool trans = false;
  int64_t nnzb = 0;
  DBuf<int64_t> own_rp;              // storage when transposed
  DBuf<int32_t> own_ci, own_blk;
};

// Index transpose of a block-CSR matrix (a0): fills op.{row_ptr,col_idx,blk}
// with the block-CSR of X^T, entries of each new row in ascending old row.
void transpose_index(Allocator &al, const bsmm_mat_s &x, OpIndex &op, hipStream_t s);

// Frobenius norm of every block (a1).
void block_norms(const bsmm_mat_s &x, double *norms, hipStream_t s);

// Sizes the plan reads back, gathered in one 8-entry record (one copy to
// the host): out[0..3] = *at[0..3], out[4..6] = the sums of sum[0..2] over
// n entries, out[7] = the largest of mx64[0..nmx) or mx32[0..nmx) (0 if
// neither); a null pointer reads as 0.
struct PlanTotals {
  const int64_t *at[4] = {nullptr, nullptr, nullptr, nullptr};
  const int64_t *sum[3] = {nullptr, nullptr, nullptr};
  int64_t n = 0;
  const int64_t *mx64 = nullptr;
  const int32_t *mx32 = nullptr;
  int64_t nmx = 0;
};
void plan_totals(const PlanTotals &T, int64_t *out, hipStream_t s);

struct SymArgs {
  const OpIndex *a, *b;
  // C_old pattern (may be null)
  const int64_t *cold_rp = nullptr;
  const int32_t *cold_ci = nullptr;
  bool use_cold = false;     // include C_old pattern (beta != 0 && !retain)
  bool retain = false;       // pattern = C_old pattern exactly
  int32_t nbc = 0;           // block columns of C
  const int32_t *ord = nullptr;   // order in which rows are handed out (device; null = 0..nbr-1)
  uint32_t *bits = nullptr;       // per-row column bitmaps kept from count to fill (optional,
                                  // symbolic_bits_words(nbr, nbc) words)
};

// Words of the per-row bitmaps the counting pass can keep for the fill; 0
// when the columns need several bitmap windows or the bitmaps would be large.
size_t symbolic_bits_words(int32_t nbr, int32_t nbc);

// a2: per C block row, number of distinct result block columns (max_row:
// optional, receives the largest by atomics).
void symbolic_count(const SymArgs &g, int64_t *row_nnz, int32_t *max_row, hipStream_t s);

struct FillArgs {
  SymArgs sym;
  const int64_t *c_rp = nullptr;   // C row_ptr (from the scan)
  int32_t *c_ci = nullptr;         // out: C col_idx
  int32_t *c_row = nullptr;        // out: block row of every C block
  int64_t *c_size = nullptr;       // out: m*n of every C block
  int32_t *c_cnt = nullptr;        // out: kept products per C block (zeroed before)
  int64_t *c_kflops = nullptr;     // out: per block row, sum of m*k*n over kept products
  int64_t *row_cand = nullptr;     // out: per block row, candidate products (before filters)
  int64_t *row_real = nullptr;     // out: per block row, kept products (without padding)
  bool pad4 = false;               // pad every equal-k-size run of a segment to 4 entries
  std::vector<int32_t> ksizes;     // distinct k block sizes, ascending (when pad4)
  int32_t *cnt_g = nullptr;        // nnzb_C * |ksizes| zeroed counters for wide rows
  int32_t *kofs = nullptr;         // out (when pad4): start of every k-size run inside its
                                   // C block's segment, nnzb_C * |ksizes| entries
  bool diag8 = false;              // pad runs of blocks with both edges <= 8 to groups of eight
  const double *na = nullptr;      // norms of A's blocks (null when eps == 0)
  const int4 *bent = nullptr;      // product records of op(B) (product_records)
  double eps = 0.0;
  int32_t max_row = 0;
  // out (optional, 2 doubles preset to +inf and 0): the smallest kept and the
  // largest dropped norm product of the on-the-fly filter
  double *margin = nullptr;
};

// a2 (fill) + a4 (count): C col_idx, block sizes, product counts.
void symbolic_fill(const FillArgs &f, hipStream_t s);

// Column windows of the stack generator: window w holds block columns
// [w*wc, (w+1)*wc).  nwin = 0: no windows (one pass per row and k size).
// Per-row counters (result blocks x k sizes) the symbolic fill keeps in LDS;
// wider rows count in global memory (a zeroed array of that many per block).
constexpr int32_t SYM_CNT_CAP = 16384;

struct StackWindows {
  int nwin = 0;
  int32_t wc = 0;
};

// Windows for a product with nbc block columns whose widest result row has
// max_row blocks, nks k sizes; nwin = 0 where the windowed generator does
// not apply (it needs the quad path's k-size runs, a bitmap window and
// windows whose result blocks fit its LDS).
StackWindows stack_windows(int32_t nbc, int32_t max_row, int nks);

// out[r*(nwin+1) + w] = first entry of row r with column >= w*wc (the row's
// end for w = nwin); row_max (optional, nrows entries) receives for every
// row the largest number of its entries inside one window.
void window_bounds(const int64_t *rp, const int32_t *ci, int32_t nrows, const StackWindows &sw, int64_t *out,
                   int32_t *row_max, hipStream_t s);

struct StackArgs {
  const OpIndex *a, *b;
  const int64_t *c_rp = nullptr;
  const int32_t *c_ci = nullptr;
  const int64_t *seg_off = nullptr;  // start of every C block's stack segment
  int2 *stack = nullptr;             // out: (a_blk, b_blk)
  const double *na = nullptr;        // norms of op(A)'s blocks (null: no filter)
  double eps = 0.0;
  int32_t nbc = 0;
  int32_t nbr = 0;
  int32_t max_row = 0;
  std::vector<int32_t> ksizes;       // distinct k block sizes, ascending
  bool pad4 = false;                 // pad every equal-k-size run to 4 entries (null = -1)
  bool encode = false;               // entries = byte offsets | (k-1) bits (quad path), null = 0x80000000
  const int32_t *kofs = nullptr;     // k-size run starts inside each segment (pad4)
  const int64_t *a_poff = nullptr;   // packed block offsets of A used by the encoded entries
  const int64_t *a_base = nullptr;   // per row of op(A): offset the encoded A offsets are taken from (null: 0)
  const int4 *bent = nullptr;        // product records of op(B) (product_records)
  StackWindows win;                  // windowed generation when win.nwin > 0:
  const int64_t *wslot = nullptr;    //   window bounds of C's rows
  const int64_t *bwin = nullptr;     //   window bounds of op(B)'s rows
  int32_t max_ns = 0;                //   most C blocks of one row in one window
  const int32_t *ord = nullptr;      // order in which rows are handed out (device; null = 0..nbr-1)
  bool diag8 = false;                // runs of blocks with both edges <= 8 padded to groups of eight
};

// Per entry of op(B), one 16-byte record read by the symbolic fill and the
// stack generator: block column, the B half of a stack entry (byte offset
// into the packed copy of op(B) when b_poff is given -- from the start of
// its column's packed blocks when b_base is given too -- else the block id)
// and the block norm (0 when nb is null).
void product_records(const OpIndex &b, const double *nb, const int64_t *b_poff, const int64_t *b_base, int4 *out,
                     hipStream_t s);

// Sets *flag (preset to 0) when some candidate product of op(A) x op(B) is
// kept under one set of block norms and dropped under the other (norms
// indexed by stored block id).
void decisions_differ(const OpIndex &a, const OpIndex &b, const double *na0, const double *nb0, const double *na1,
                      const double *nb1, double eps, int32_t *flag, hipStream_t s);

// a4: stack entries, grouped by C block, ascending k inside a block.  `run`
// (nnzb of C, zeroed) serves rows too wide for the LDS cursors.
void stack_fill(const StackArgs &g, int32_t *run, hipStream_t s);

// For every C_old block, store its id at the matching C block (old_blk must
// be preset to -1).
void old_block_map(const int64_t *cold_rp, const int32_t *cold_ci, int32_t nbr, const int64_t *c_rp,
                   const int32_t *c_ci, int32_t *old_blk, hipStream_t s);

// Per work item of the GEMM (one C block, in work-list order): everything a
// wavefront needs before its first stack round, in one 32-byte record.
struct alignas(32) BlkDesc {
  int32_t c;    // C block id
  int32_t mn;   // m | n << 16 (block edges)
  int64_t s0;   // first stack entry of the block's segment
  int64_t co;   // value offset of the C block
  int32_t ns;   // stack entries of the segment
  int32_t pad;
};

// Per work item, with per-unit addressing of the packed copies only: where
// the stack entries' operand offsets start (values into the packed copies),
// the packed blocks of the C block's row of op(A) and of its column of op(B).
struct alignas(16) UnitBases {
  int64_t a, b;
};

// Workgroups of a GEMM launch to XCDs.  The hardware deals workgroup ids to
// the 8 XCDs round-robin; the kernels remap them so that the XCDs take
// chunks of `chunk` consecutive work items in turn, all working on
// neighbouring tiles of the work list at once (their shared infinity cache
// sees the same operands).  per_xcd (workgroups per XCD) is a multiple of
// chunk, so the remap is a bijection onto [0, 8 * per_xcd); ids past the
// last work item exit.  Small launches get one chunk per XCD.
struct XcdMap {
  int64_t per_xcd = 0, chunk = 1;
};
inline XcdMap xcd_map(int64_t nwg, int64_t max_chunk = 8192) {
  XcdMap m;
  const int64_t base = (nwg + 7) / 8;
  m.chunk = std::max<int64_t>(1, std::min(max_chunk, base));
  m.per_xcd = (base + m.chunk - 1) / m.chunk * m.chunk;
  return m;
}
__device__ __forceinline__ int64_t xcd_logical(int64_t b, int64_t chunk) {
  const int64_t g = b >> 3;
  return (g / chunk) * (8 * chunk) + (b & 7) * chunk + g % chunk;
}

struct GemmArgs {
  const OpIndex *a, *b;
  const int32_t *c_list = nullptr;   // C blocks ordered by class
  const BlkDesc *desc = nullptr;     // work-item descriptors (quad path)
  const UnitBases *ubase = nullptr;  // per work item, per-unit addressing only (else offsets from each copy's start)
  const int32_t *c_row = nullptr;
  const int32_t *c_ci = nullptr;
  const int64_t *c_off = nullptr;    // value offsets of C blocks
  const int64_t *seg_off = nullptr;
  const int2 *stack = nullptr;
  const int32_t *c_old_blk = nullptr;
  const int64_t *old_off = nullptr;
  const double *old_values = nullptr;
  double *c_values = nullptr;
  double *c_norm = nullptr;          // out: norm of every C block (may be null)
  double alpha = 1.0, beta = 0.0;
  bsmm_compute_mode mode = BSMM_COMPUTE_FP64;
  const double *a_cm = nullptr;      // op(A) blocks, column-major (m x K) (walker path)
  const double *b_rm = nullptr;      // op(B) blocks, row-major (K x n) (walker path)
  const double *a_pack = nullptr;    // packed op(A): row-major, k padded to even (quad path)
  const double *b_pack = nullptr;    // packed op(B): column-major, k padded to even (quad path)
  const float *a_hi = nullptr, *a_lo = nullptr;   // packed FP32 k-quad slabs (FP32 / split modes)
  const float *b_hi = nullptr, *b_lo = nullptr;
  uint64_t a_bytes = 0, b_bytes = 0; // sizes of the two value arrays the kernel reads
  bool quads = false;                // stacks padded to k-homogeneous quads (quad path)
  uint8_t variant[16] = {};          // GEMM kernel variant per (m, n) size class
  const double *zeros = nullptr;     // >= 4 KB of zeros
};

// *flag |= 1 when x and y differ somewhere in their first n entries.
void differs_i64(const int64_t *x, const int64_t *y, int64_t n, int32_t *flag, hipStream_t s);
void differs_i32(const int32_t *x, const int32_t *y, int64_t n, int32_t *flag, hipStream_t s);
// p[t] = a for even t, b for odd t, t < n <= 64.
void set_pairs(double *p, int n, double a, double b, hipStream_t s);
// out[0] = min(out[0], now[t] / then[t]), out[1] = max(out[1], ...) over t < n
// (out preset to +inf, 0); a ratio that is not finite gives 0 and +inf.
void ratio_bounds(const double *then, const double *now, int64_t n, double *out, hipStream_t s);

// out[t] = t for t < n.
void fill_sequence(int32_t *out, int32_t n, hipStream_t s);

// Block-diagonal identity values (block i of size sizes[i] at off[i]).
void identity_values(const int32_t *d_sizes, const int64_t *d_off, int32_t n, double *values, hipStream_t s);
// row_out[i] = sum over block row i of ||X_ij - shift * delta_ij I||_F^2 (square x).
void shift_dist_rows(const bsmm_mat_s &x, double shift, double *row_out, hipStream_t s);

// Packed operand copies (quad path): per stored block, nr rows of
// Kp = K + (K & 1) values contiguous in k (pad zero).  k_is_row: the block's
// row count is the contraction extent (op(A) = A^T or op(B) = B).
// pack_offsets writes nnzb + 1 offsets (exclusive scan, total last).
void pack_offsets(Allocator &al, const bsmm_mat_s &x, bool k_is_row, int64_t *d_poff, hipStream_t s);
// The same offsets laid out unit by unit: the rows of `units` are the units
// (the rows of op(A), or the columns of op(B)), each listing the positions
// of its blocks in x's storage (units.blk; identity when null), and every
// unit's packed blocks are contiguous.  base[r] (units.nbr entries) is the
// offset of unit r's first block, so a block's offset minus its unit's base
// stays below the unit's packed size.
void pack_offsets_units(Allocator &al, const bsmm_mat_s &x, bool k_is_row, const OpIndex &units, int64_t *d_poff,
                        int64_t *d_base, hipStream_t s);
// Both packed operand copies in one launch; with a_norm / b_norm, the block
// norms as well, bitwise equal to block_norms (same summation order).
void pack_values(const bsmm_mat_s &a, bool a_k_is_row, const int64_t *a_poff, double *a_out, const bsmm_mat_s &b,
                 bool b_k_is_row, const int64_t *b_poff, double *b_out, hipStream_t s, double *a_norm = nullptr,
                 double *b_norm = nullptr);
// FP32 k-quad slabs (FP32 / split modes): offsets in units of 8 bytes; lo
// (the rounding remainder x - fp32(x)) is written only when non-null.
void pack32_offsets(Allocator &al, const bsmm_mat_s &x, bool k_is_row, int64_t *d_poff, hipStream_t s);
void pack32_values(const bsmm_mat_s &x, bool k_is_row, const int64_t *d_poff, float *hi, float *lo, hipStream_t s);
// a5 in FP32 or split-FP32 arithmetic (g.mode), quad path only.
void gemm_launch_lowp(const GemmArgs &g, int64_t nnzb_c, int max_edge, hipStream_t s);

// Transpose every stored block of x into out (same offsets).
void transpose_blocks(const bsmm_mat_s &x, double *out, hipStream_t s);

// a5: batched small-GEMM over the stacks, one launch over all C blocks in
// c_list order (max_edge: largest C block edge).
void gemm_launch(const GemmArgs &g, int64_t nnzb_c, int max_edge, hipStream_t s);

// a5 for several multiplications in one launch (packed-operand FP64 path):
// the parameter blocks go through h_stage (pinned host) to d_stage (device),
// both stage_bytes large; the caller keeps d_stage untouched until the
// launch has finished.
void gemm_launch_multi(Allocator &al, const std::vector<const GemmArgs *> &gs, const std::vector<int64_t> &nnzb,
                       int max_edge, void *h_stage, size_t stage_bytes, void *d_stage, hipStream_t s);
size_t gemm_multi_stage_bytes(int n);   // staging bytes for n requests

// Unit bases of the packed operands (per-unit addressing): out[w] receives
// those of work item w's row of op(A) and column of op(B); all null without.
struct DescBases {
  const int64_t *a = nullptr;   // per row of op(A)
  const int64_t *b = nullptr;   // per column of op(B)
  UnitBases *out = nullptr;     // per work item
};

// desc[w] for the work items w < n (C block c_list[w], or w without a list).
void build_desc(int64_t n, const int32_t *c_list, const int32_t *c_row, const int32_t *c_ci, const int32_t *rbs,
                const int32_t *cbs, const int64_t *seg, const int64_t *c_off, DescBases bases, BlkDesc *desc,
                hipStream_t s);

// c_list = C blocks in tiles of consecutive rows of ord (device), column by
// column inside a tile.
void build_work_list(Allocator &al, const int32_t *d_ord, const int32_t *d_rank, const int64_t *c_rp,
                     const int32_t *c_ci, int32_t nbr, int32_t nbc, int32_t tile_rows, int32_t *c_list, hipStream_t s);

// c_list = the C blocks sorted by (tile of their row, rank of their column):
// tiles of tile_rows (a multiple of 16) consecutive rows of the locality
// order ord, columns by crank (null: by index).  Needs nbc int32 counters in
// LDS and ceil(nbr / tile_rows) * nbc * tile_rows / 16 keys in memory.
// pos (optional, nnzb_c entries) receives the place of every C block in
// the list (the inverse of c_list).
void build_work_list_sorted(Allocator &al, const int32_t *ord, const int32_t *crank, const int64_t *c_rp,
                            const int32_t *c_ci, int64_t nnzb_c, int32_t nbr, int32_t nbc, int32_t tile_rows,
                            int32_t *c_list, int32_t *pos, hipStream_t s);

// desc[pos[c]] for every C block c < n (as build_desc, from the inverse of
// the work list).
void build_desc_by_block(int64_t n, const int32_t *pos, const int32_t *c_row, const int32_t *c_ci, const int32_t *rbs,
                         const int32_t *cbs, const int64_t *seg, const int64_t *c_off, DescBases bases,
                         BlkDesc *desc, hipStream_t s);

// ---------------------------------------------------- tile path of the GEMM
// Result blocks in tiles of ti x tj (rows adjacent in the locality order,
// columns too); one workgroup per tile, (ti/2)(tj/2) wavefronts each owning
// a 2 x 2 part of it; the operand blocks the tile uses at a k are staged in
// LDS once for all its products.
struct TileShape {
  int ti = 2, tj = 2;
};
// Descriptors and step records of a product's tiles (layouts depend on the
// shape; see tile_gemm.hip).
struct TilePlan {
  TileShape sh;
  int64_t ntile = 0, nsteps = 0;
  DBuf<int4> tiles, steps;
};
struct TileArgs {
  const int32_t *rbs = nullptr, *cbs = nullptr;   // C block sizes
  const double *a_val = nullptr, *b_val = nullptr;
  int64_t a_n = 0, b_n = 0;   // stored values of A and B
  bool ta = false, tb = false;
  const int64_t *c_off = nullptr;
  const int32_t *old_blk = nullptr;
  const int64_t *old_off = nullptr;
  const double *old_val = nullptr;
  double *c_val = nullptr;
  double *c_norm = nullptr;
  double alpha = 1.0, beta = 0.0;
  int32_t uni = 0;   // S when every block of op(A), op(B) and C is S x S and a kernel for S exists (2 x 2 tiles)
  int64_t xcd_chunk = 0;   // tiles per XCD chunk (0: 8192)
};
// Tile shapes the kernels are built for.
bool tile_shape_valid(int ti, int tj);
// Whether a uniform-size tile kernel exists for S x S blocks.
bool tile_uni_size(int32_t sz);
// Whether the tile plan's LDS bitmaps hold a product with nbc block columns
// of C and nbk contraction blocks.
bool tile_path_fits(int32_t nbc, int32_t nbk, TileShape sh);
// The rows of op(A): row pointers, block columns (k) and stored block ids
// (null: the positions) of its entries.
struct OpRows {
  const int64_t *rp = nullptr;
  const int32_t *ci = nullptr;
  const int32_t *blk = nullptr;
  int64_t nnzb = 0;
};
// The one block area of A and of B (0: blocks of several areas) and their
// numbers of stored blocks: with one area, block p starts at p times it
// (blocks are stored in order), which the tile plan checks and then uses.
struct OffsetAreas {
  int64_t a_area = 0, b_area = 0;
  int64_t a_n = 0, b_n = 0;
};
// Tiles of the result pattern (rows grouped in the order ord, null =
// natural; columns by crank, null = natural, cinv its inverse) and their step
// records from the per-result-block stacks (entries = stored A and B block
// ids, ascending k; ar: the rows of op(A), nbk its block columns): two host
// synchronisations for the sizes.
void build_tile_plan(Allocator &al, TileShape sh, const int32_t *ord, const int32_t *crank, const int32_t *cinv,
                     int32_t nbr, int32_t nbc, const int64_t *c_rp, const int32_t *c_ci, const int64_t *seg,
                     const int2 *stack, const OpRows &ar, int32_t nbk, const int32_t *ksz, const int64_t *a_off,
                     const int64_t *b_off, OffsetAreas ob, int64_t *pinned, TilePlan &tp, hipStream_t s);
// a5 on the tile path.
void tile_gemm_launch(const TilePlan &tp, const TileArgs &g, hipStream_t s);

// Takes the device address of the allocation-free filter's scratch array on
// `device` (the current device), once per device.
void noalloc_init(int device);

// Locality order of the rows of a square block pattern (host planner).
std::vector<int32_t> locality_order(int32_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci);

// a6: keep flags from norms, compaction of a block-CSR matrix.
struct CompactArgs {
  int32_t nbr = 0;
  int64_t nnzb = 0;
  const int64_t *rp = nullptr;
  const int32_t *ci = nullptr;
  const int64_t *off = nullptr;
  const double *values = nullptr;
  const double *norm = nullptr;
  double eps = 0.0;
};
// Returns the number of kept blocks (synchronises to read it back).  When
// every block is kept nothing is written and the caller keeps its arrays.
int64_t count_kept(Allocator &al, const CompactArgs &c, int32_t *keep_prefix_tmp, int64_t *pinned,
                   hipStream_t s, DBuf<int64_t> &new_rank);
// Values go to dst when given (room for the kept values; it must not overlap
// c.values), else to a new allocation.
void compact(Allocator &al, const CompactArgs &c, const int64_t *new_rank, const int32_t *d_rbs,
             const int32_t *d_cbs, int64_t *new_rp, int32_t *new_ci, int64_t *new_off,
             int64_t *pinned, double **new_values, int64_t *new_nval, hipStream_t s, double *dst = nullptr);

}  // namespace bsmm
