// api.hip -- the C ABI of libbsmm: contexts, matrices, norms, multiply and
// filter.  Host code only: validation, sizing, phase sequencing on the
// context stream; every step of the multiply runs in the library's kernels.
#include <algorithm>
#include <cstring>
#include <new>
#include <sstream>

#include "internal.h"

namespace bsmm {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(bsmm_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e == hipSuccess) return;
  std::ostringstream os;
  os << what << " failed: " << hipGetErrorString(e) << " (" << file << ":" << line << ")";
  if (e == hipErrorOutOfMemory) fail(BSMM_ERR_OUT_OF_MEMORY, os.str());
  fail(BSMM_ERR_DEVICE, os.str());
}

// ----------------------------------------------------------------- allocator
static size_t round_up(size_t b) {
  const size_t g = 256;
  if (b == 0) b = 1;
  return (b + g - 1) / g * g;
}

void Allocator::init(int device, size_t budget) {
  device_ = device;
  budget_ = budget;
}

void *Allocator::alloc(size_t bytes) {
  size_t sz = round_up(bytes);
  // reuse a cached block of at most twice the size
  auto it = free_.lower_bound(sz);
  if (it != free_.end() && it->first <= 2 * sz) {
    void *p = it->second;
    size_t have = it->first;
    free_.erase(it);
    cached_ -= have;
    live_[p] = have;
    return p;
  }
  if (budget_ && held_ + sz > budget_) {
    trim();
    if (held_ + sz > budget_) {
      std::ostringstream os;
      os << "allocation of " << sz << " bytes exceeds the context budget (" << budget_ << " bytes, "
         << held_ << " held)";
      fail(BSMM_ERR_OUT_OF_MEMORY, os.str());
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim();
    e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      std::ostringstream os;
      os << "hipMalloc of " << sz << " bytes failed";
      fail(BSMM_ERR_OUT_OF_MEMORY, os.str());
    }
  }
  held_ += sz;
  peak_ = std::max(peak_, held_);
  live_[p] = sz;
  return p;
}

void Allocator::release(void *p) {
  if (!p) return;
  auto it = live_.find(p);
  if (it == live_.end()) return;
  free_.emplace(it->second, p);
  cached_ += it->second;
  live_.erase(it);
}

void Allocator::trim() {
  if (free_.empty()) return;
  // pending work may still use cached blocks: wait before freeing them
  (void)hipDeviceSynchronize();
  for (auto &kv : free_) {
    (void)hipFree(kv.second);
    held_ -= kv.first;
  }
  free_.clear();
  cached_ = 0;
}

void Allocator::check(size_t bytes, const char *what) const {
  if (!budget_) return;
  const size_t live = held_ - cached_;
  if (live + bytes > budget_) {
    std::ostringstream os;
    os << what << " needs " << bytes << " bytes beyond the " << live << " in use; the context budget is " << budget_
       << " bytes";
    fail(BSMM_ERR_OUT_OF_MEMORY, os.str());
  }
}

size_t Allocator::room() const {
  if (!budget_) return SIZE_MAX;
  const size_t live = held_ - cached_;
  return live < budget_ ? budget_ - live : 0;
}

Allocator::~Allocator() {
  (void)hipDeviceSynchronize();
  for (auto &kv : free_) (void)hipFree(kv.second);
  for (auto &kv : live_) (void)hipFree(kv.first);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) HIPCHECK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

static void upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes) HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}

static constexpr int32_t MAX_BLOCK = 32;

// Owned index arrays of a matrix built inside the library.
static bsmm_mat_s *new_result(bsmm_ctx ctx, int32_t nbr, int32_t nbc, const std::vector<int32_t> &rbs,
                              const std::vector<int32_t> &cbs) {
  auto *m = new bsmm_mat_s();
  m->ctx = ctx;
  m->nbr = nbr;
  m->nbc = nbc;
  m->h_rbs = rbs;
  m->h_cbs = cbs;
  Allocator &al = ctx->alloc;
  try {
    m->d_rbs = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<size_t>(nbr, 1)));
    m->d_cbs = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<size_t>(nbc, 1)));
    upload(m->d_rbs, rbs.data(), sizeof(int32_t) * nbr, ctx->stream);
    upload(m->d_cbs, cbs.data(), sizeof(int32_t) * nbc, ctx->stream);
  } catch (...) {
    al.release(m->d_rbs);
    al.release(m->d_cbs);
    delete m;
    throw;
  }
  m->owns_values = true;
  return m;
}

static void free_mat(bsmm_mat_s *m) {
  Allocator &al = m->ctx->alloc;
  al.release(m->d_rbs);
  al.release(m->d_cbs);
  al.release(m->d_row_ptr);
  al.release(m->d_col_idx);
  al.release(m->d_blk_off);
  al.release(m->d_order);
  if (m->owns_values) al.release(m->d_values);
  delete m;
}

// Locality order of x's block rows for the GEMM work list, computed once per
// matrix from its (immutable) block pattern and cached on the device: nbr
// entries of the order, then nbr entries of its inverse (the rank of a row,
// also used for the columns of a square product).
// Locality order of a square operand's block rows (computed on the host
// once per matrix, then cached).  Automatic mode skips operands of fewer than
// ROW_ORDER_MIN block rows: the order costs a pattern read-back and a host
// bisection for every new matrix (1 to 25 ms between 300 and 3,000 rows)
// and, measured on DFT-like operands of 300 to 3,000 atoms, did not speed up
// their GEMM, while 4,000 to 8,000 atoms gain 19 to 27 %.
constexpr int32_t ROW_ORDER_MIN = 2048;
static const int32_t *row_order(bsmm_ctx ctx, bsmm_mat_s *x) {
  if (ctx->row_order == 2) return nullptr;
  if (x->d_order) return x->d_order;
  if (x->nbr != x->nbc || x->nbr < (ctx->row_order == 1 ? 64 : ROW_ORDER_MIN)) return nullptr;
  std::vector<int64_t> rp((size_t)x->nbr + 1);
  std::vector<int32_t> ci((size_t)std::max<int64_t>(x->nnzb, 1));
  HIPCHECK(hipMemcpyAsync(rp.data(), x->d_row_ptr, sizeof(int64_t) * rp.size(), hipMemcpyDeviceToHost, ctx->stream));
  if (x->nnzb)
    HIPCHECK(hipMemcpyAsync(ci.data(), x->d_col_idx, sizeof(int32_t) * (size_t)x->nnzb, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  x->h_order = locality_order(x->nbr, rp, ci);
  x->h_order.resize(2 * (size_t)x->nbr);
  for (int32_t r = 0; r < x->nbr; r++) x->h_order[(size_t)x->nbr + x->h_order[r]] = r;
  x->d_order = static_cast<int32_t *>(ctx->alloc.alloc(sizeof(int32_t) * 2 * (size_t)x->nbr));
  HIPCHECK(hipMemcpyAsync(x->d_order, x->h_order.data(), sizeof(int32_t) * 2 * (size_t)x->nbr, hipMemcpyHostToDevice,
                          ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  return x->d_order;
}

// The area of x's blocks when they all have one (every row and every column
// block size the same), else 0.
static int64_t one_block_area(const bsmm_mat_s *x) {
  if (x->h_rbs.empty() || x->h_cbs.empty()) return 0;
  for (int32_t r : x->h_rbs)
    if (r != x->h_rbs[0]) return 0;
  for (int32_t c : x->h_cbs)
    if (c != x->h_cbs[0]) return 0;
  return (int64_t)x->h_rbs[0] * x->h_cbs[0];
}

static void make_op(bsmm_ctx ctx, bsmm_mat_s *x, bool trans, OpIndex &op) {
  op.blk_off = x->d_blk_off;
  op.values = x->d_values;
  if (!trans) {
    op.nbr = x->nbr;
    op.nbc = x->nbc;
    op.nnzb = x->nnzb;
    op.row_ptr = x->d_row_ptr;
    op.col_idx = x->d_col_idx;
    op.blk = nullptr;
    op.rbs = x->d_rbs;
    op.cbs = x->d_cbs;
    op.trans = false;
  } else {
    transpose_index(ctx->alloc, *x, op, ctx->stream);
    op.rbs = x->d_cbs;
    op.cbs = x->d_rbs;
  }
}

struct Timer {
  bsmm_ctx ctx;
  std::vector<hipEvent_t> ev;
  explicit Timer(bsmm_ctx c) : ctx(c) {}
  void mark() {
    if (!ctx->timing) return;
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, ctx->stream));
    ev.push_back(e);
  }
  float between(size_t a, size_t b) {
    if (!ctx->timing || b >= ev.size()) return 0.f;
    HIPCHECK(hipEventSynchronize(ev[b]));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, ev[a], ev[b]));
    return ms;
  }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// One multiplication, split into its structural part (validation, index
// views, norms, symbolic phase, stacks, work list, every buffer of the
// numeric part), its numeric part (packed operand copies and the block GEMM:
// kernels only -- no host synchronisation, allocation or memset, so it can
// be captured in a HIP graph and replayed while the values of A, B and C_old
// change) and the post-filter that sizes and assembles the result.  The
// filter decisions of the stacks are taken on the values A and B have when
// the plan is built.
struct Plan {
  bsmm_ctx ctx = nullptr;
  bsmm_mat_s *A = nullptr, *B = nullptr, *C0 = nullptr;
  bool ta = false, tb = false, filt = false, post = false, quads = false, lowp = false, tiles = false;
  // packed path with per-unit addressing: stack entries hold offsets from
  // the start of their op(A) row's / op(B) column's packed blocks (a_base,
  // b_base), so the copies may exceed 2 GB
  bool units = false;
  int32_t uni = 0;   // block size of the uniform-size tile kernel (0: the general one)
  // one_shot: built, executed once and consumed (bsmm_multiply); packed:
  // plan_build already made the packed operand copies of the current values
  bool one_shot = false, packed = false;
  double alpha = 1.0, beta = 0.0, eps = 0.0;
  int retain = 0;
  bsmm_compute_mode mode = BSMM_COMPUTE_FP64;
  int32_t nbr = 0, nbc = 0, max_edge = 1;
  std::vector<int32_t> opa_r, opb_c;
  int64_t nnzb_c = 0, nval_c = 0, nstack = 0, nprod = 0, kmn_total = 0, ncand = 0;
  int64_t a_pack_n = 0, b_pack_n = 0;
  OpIndex oa, ob;
  DBuf<int64_t> c_rp, c_off, seg_off, a_poff, b_poff, a_base, b_base;
  DBuf<int32_t> c_ci, c_row, old_blk, c_list;
  DBuf<BlkDesc> desc;
  DBuf<UnitBases> ubase;   // per work item, per-unit addressing only
  DBuf<int2> stack;
  DBuf<double> a_pack, b_pack, a_lo, b_lo, a_t, b_t, c_norm, c_values;
  GemmArgs ga;
  // Buffers of the numeric part.  A plan computes their layout; they are
  // either library-owned (own_cval, own_ws: allocated by the first execution)
  // or the caller's (bsmm_plan_execute_into).  Workspace regions, byte
  // offsets from its start, 256-byte aligned: packed op(A) and op(B) (and
  // their low parts in split mode), transposed operand copies of the walker
  // path, result-block norms and, with a post-filter, a copy of the result
  // values the compaction reads from.
  struct Ws {
    size_t apack = 0, bpack = 0, alo = 0, blo = 0, at = 0, bt = 0, cnorm = 0, stash = 0, total = 0;
    size_t core = 0;   // bytes before the stash (all a library-owned execution needs)
    bool has_apack = false, has_alo = false, has_at = false, has_bt = false, has_cnorm = false;
  } ws;
  DBuf<double> own_cval;
  DBuf<uint8_t> own_ws;
  double *cval = nullptr;     // bound result values (nval_c)
  uint8_t *wsp = nullptr;     // bound workspace
  bool bound = false, caller_bound = false;
  // filter decisions of a reusable plan: the block norms they were taken
  // on and the smallest kept / largest dropped norm product (device)
  DBuf<double> na_plan, nb_plan, margin;
  // tile path: tiles of result blocks and their per-k step records
  TilePlan tp;
  TileArgs targs;
  Timer tm;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  explicit Plan(bsmm_ctx c) : ctx(c), tm(c) {}
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// Points the numeric part at result values cval (nval_c doubles) and the
// workspace wsp (P.ws.total bytes, 256-byte aligned).
static void bind_numeric(Plan &P, double *cval, uint8_t *wsp) {
  const Plan::Ws &w = P.ws;
  auto at = [&](size_t o, bool has) { return has ? reinterpret_cast<double *>(wsp + o) : nullptr; };
  double *apack = at(w.apack, w.has_apack), *bpack = at(w.bpack, w.has_apack);
  double *alo = at(w.alo, w.has_alo), *blo = at(w.blo, w.has_alo);
  double *a_t = at(w.at, w.has_at), *b_t = at(w.bt, w.has_bt);
  double *cnorm = at(w.cnorm, w.has_cnorm);
  GemmArgs &ga = P.ga;
  ga.c_values = cval;
  ga.c_norm = cnorm;
  // operand layouts: packed copies (quad path), or op(A) column-major and
  // op(B) row-major (walker path)
  ga.a_cm = P.ta ? a_t : P.A->d_values;
  ga.b_rm = P.tb ? P.B->d_values : b_t;
  ga.a_pack = apack;
  ga.b_pack = bpack;
  ga.a_hi = reinterpret_cast<const float *>(apack);
  ga.b_hi = reinterpret_cast<const float *>(bpack);
  ga.a_lo = reinterpret_cast<const float *>(alo);
  ga.b_lo = reinterpret_cast<const float *>(blo);
  P.targs.c_val = cval;
  P.targs.c_norm = cnorm;
  P.cval = cval;
  P.wsp = wsp;
  P.bound = true;
}

// One-shot product whose packing kernel already wrote the packed copies
// (with the norms) into P.a_pack / P.b_pack.
static void bind_packed(Plan &P) {
  GemmArgs &ga = P.ga;
  ga.c_values = P.c_values.p;
  ga.c_norm = P.post ? P.c_norm.p : nullptr;
  ga.a_cm = P.A->d_values;
  ga.b_rm = P.B->d_values;
  ga.a_pack = P.a_pack.p;
  ga.b_pack = P.b_pack.p;
  ga.a_hi = reinterpret_cast<const float *>(P.a_pack.p);
  ga.b_hi = reinterpret_cast<const float *>(P.b_pack.p);
  ga.a_lo = ga.b_lo = nullptr;
  P.targs.c_val = P.c_values.p;
  P.targs.c_norm = ga.c_norm;
  P.cval = P.c_values.p;
  P.bound = true;
}

// Library-owned buffers of the numeric part, allocated (within the budget,
// before any kernel of the calling operation) the first time a plan runs
// without caller buffers.
static void ensure_own_buffers(Plan &P) {
  if (P.bound && !P.caller_bound) return;
  Allocator &al = P.ctx->alloc;
  if (!P.own_cval.p) P.own_cval = DBuf<double>(al, (size_t)std::max<int64_t>(P.nval_c, 1));
  if (!P.own_ws.p) P.own_ws = DBuf<uint8_t>(al, std::max<size_t>(P.ws.core, 256));
  bind_numeric(P, P.own_cval.p, P.own_ws.p);
  P.caller_bound = false;
}

static void plan_build(Plan &P, char transa, char transb) {
  bsmm_ctx ctx = P.ctx;
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  bsmm_mat_s *A = P.A, *B = P.B, *C0 = P.C0;
  const double beta = P.beta, eps = P.eps;
  const int retain = P.retain;
  const bool ta = P.ta = (transa == 'T' || transa == 't');
  const bool tb = P.tb = (transb == 'T' || transb == 't');
  // ---------------------------------------------------------- validation
  const std::vector<int32_t> &opa_r = ta ? A->h_cbs : A->h_rbs;
  const std::vector<int32_t> &opa_c = ta ? A->h_rbs : A->h_cbs;
  const std::vector<int32_t> &opb_r = tb ? B->h_cbs : B->h_rbs;
  const std::vector<int32_t> &opb_c = tb ? B->h_rbs : B->h_cbs;
  if (opa_c.size() != opb_r.size()) fail(BSMM_ERR_SHAPE, "op(A) block columns != op(B) block rows");
  for (size_t k = 0; k < opa_c.size(); k++)
    if (opa_c[k] != opb_r[k]) fail(BSMM_ERR_SHAPE, "op(A) column block sizes differ from op(B) row block sizes");
  for (int32_t v : opa_r) if (v > MAX_BLOCK) fail(BSMM_ERR_UNSUPPORTED, "block sizes above 32 are not supported");
  for (int32_t v : opb_c) if (v > MAX_BLOCK) fail(BSMM_ERR_UNSUPPORTED, "block sizes above 32 are not supported");
  for (int32_t v : opa_c) if (v > MAX_BLOCK) fail(BSMM_ERR_UNSUPPORTED, "block sizes above 32 are not supported");
  const bool need_old = (beta != 0.0) || retain;
  if (need_old && !C0) fail(BSMM_ERR_INVALID_ARG, "c_old is required when beta != 0 or retain_sparsity");
  if (C0) {
    if (C0->h_rbs != opa_r || C0->h_cbs != opb_c) fail(BSMM_ERR_SHAPE, "c_old block sizes do not match op(A) rows / op(B) columns");
    if (need_old && C0->d_values && (C0->d_values == A->d_values || C0->d_values == B->d_values) && C0->n_values > 0)
      fail(BSMM_ERR_ALIAS, "c_old values alias an operand");
  }
  if (!(eps >= 0.0)) fail(BSMM_ERR_INVALID_ARG, "filter_eps must be >= 0");
  const int32_t nbr = P.nbr = (int32_t)opa_r.size(), nbc = P.nbc = (int32_t)opb_c.size();
  P.opa_r = opa_r;
  P.opb_c = opb_c;
  P.mode = ctx->mode;

  Timer &tm = P.tm;
  tm.mark();  // 0
  // ------------------------------------------------------- a0: op index
  OpIndex &oa = P.oa, &ob = P.ob;
  make_op(ctx, A, ta, oa);
  make_op(ctx, B, tb, ob);
  tm.mark();  // 1
  // distinct contraction block sizes, ascending (each in 1..MAX_BLOCK,
  // checked above): a presence mask, not a sort of one entry per block
  // column -- this runs on the host while the device waits for the plan
  std::vector<int32_t> ksizes;
  {
    bool seen[MAX_BLOCK + 1] = {};
    for (int32_t v : opa_c) seen[v] = true;
    for (int32_t v = 1; v <= MAX_BLOCK; v++)
      if (seen[v]) ksizes.push_back(v);
  }
  // tile path of the GEMM (operand blocks staged in LDS per tile of result
  // blocks, read from the stored values): FP64, every edge and contraction
  // extent up to 24, and either every result block edge in 17..24 (its
  // preferred shape, unless another variant is requested for that class) or
  // operands the packed-operand path cannot take (more than 8 distinct k
  // sizes), where it replaces the pointer walker.
  // The quad (packed-operand) path takes at most 8 distinct k sizes.  Its
  // stack entries hold 32-bit byte offsets: from the start of each packed
  // copy while both copies stay below 2 GB, else (FP64) from the start of
  // their op(A) row's / op(B) column's packed blocks.  A packed block pads
  // its contraction extent k to a multiple of 2 (FP64) or 4 (FP32 / split,
  // half the bytes), so it holds at most (k + 1) / k or (k + 3) / k times the
  // values of the stored block; kmin bounds both.
  const uint64_t two_gb = 1ull << 31;
  const bool lowp = P.lowp = ctx->mode != BSMM_COMPUTE_FP64;
  const double kmin = ksizes.empty() ? 1.0 : (double)ksizes.front();
  const double grow = lowp ? 0.5 * (kmin + 3.0) / kmin : (kmin + 1.0) / kmin;
  const bool pack_ok = !ksizes.empty() && ksizes.size() <= 8 &&
                       (double)A->n_values * 8.0 * grow + 64.0 < (double)two_gb &&
                       (double)B->n_values * 8.0 * grow + 64.0 < (double)two_gb;
  // Per-unit addressing (FP64): the packed blocks of every row of op(A) and
  // every column of op(B) are contiguous and the stack entries hold offsets
  // from their start, which must stay below the 2 GB buffer range.  A unit
  // packs at most (its edge) x (sum of the padded k extents) values.
  bool units_ok = false;
  if (!lowp && !ksizes.empty() && ksizes.size() <= 8) {
    double kp = 0.0;
    for (int32_t v : opa_c) kp += (double)(v + (v & 1));
    int32_t edge = 1;
    for (int32_t v : opa_r) edge = std::max(edge, v);
    for (int32_t v : opb_c) edge = std::max(edge, v);
    units_ok = 8.0 * kp * (double)edge < (double)0x7FFFFFF0u;
  }
  bool tiles = false;
  if (!lowp && nbr > 0 && nbc > 0 && !ksizes.empty() && ksizes.back() <= 24 &&
      tile_path_fits(nbc, (int32_t)opa_c.size(), TileShape{ctx->tile_ti, ctx->tile_tj})) {
    bool all24 = true, big = true;
    for (int32_t x : opa_r) {
      all24 = all24 && x <= 24;
      big = big && x >= 17;
    }
    for (int32_t x : opb_c) {
      all24 = all24 && x <= 24;
      big = big && x >= 17;
    }
    const uint8_t v = ctx->gemm_variant[10];   // class of edges 17..24 x 17..24
    tiles = all24 && ((big && (v == 0 || v == 5 || v == 6)) || !(pack_ok || units_ok));
    // every block of op(A), op(B) and C S x S: the uniform-size kernel for S
    // (2 x 2 tiles), unless variant 6 asks for the general one
    if (tiles && v != 6 && ksizes.size() == 1 && ctx->tile_ti == 2 && ctx->tile_tj == 2 &&
        tile_uni_size(ksizes[0])) {
      bool uni = true;
      for (int32_t x : opa_r) uni = uni && x == ksizes[0];
      for (int32_t x : opb_c) uni = uni && x == ksizes[0];
      P.uni = uni ? ksizes[0] : 0;
    }
  }
  P.tiles = tiles;
  const bool quads = P.quads = !tiles && (pack_ok || units_ok);
  const bool units = P.units = quads && units_ok && (!pack_ok || ctx->pack_addr == 1);
  // ------------------------------------------------------- a1: norms
  // A one-shot FP64 product on the packed path reads A and B once: the
  // packing kernel computes the block norms as well (after the symbolic
  // count, when the packed sizes are known), bitwise equal to block_norms.
  DBuf<double> na, nb;
  const bool filt = P.filt = eps > 0.0;
  const bool fuse = P.one_shot && quads && !lowp && filt && !retain;
  if (filt) {
    na = DBuf<double>(al, std::max<int64_t>(A->nnzb, 1));
    nb = DBuf<double>(al, std::max<int64_t>(B->nnzb, 1));
    if (!fuse) {
      block_norms(*A, na.p, s);
      block_norms(*B, nb.p, s);
    }
  }
  tm.mark();  // 2
  // packed operand offsets for the quad path (op(A) row-major, op(B)
  // column-major) and one record per entry of op(B) for the product loops
  // of a2 and a4: both depend on A and B only, so they are queued before
  // the symbolic phase's size read-back and run while the host waits
  if (quads) {
    P.a_poff = DBuf<int64_t>(al, (size_t)A->nnzb + 1);
    P.b_poff = DBuf<int64_t>(al, (size_t)B->nnzb + 1);
    if (lowp) {   // FP32 k-quad slabs
      pack32_offsets(al, *A, ta, P.a_poff.p, s);
      pack32_offsets(al, *B, !tb, P.b_poff.p, s);
    } else if (units) {   // FP64 k-pair slabs, unit by unit
      // units of op(A): its rows (oa); of op(B): its columns, the stored
      // rows of B when op(B) = B^T, else the rows of B's transposed index
      P.a_base = DBuf<int64_t>(al, (size_t)std::max<int32_t>(nbr, 1));
      P.b_base = DBuf<int64_t>(al, (size_t)std::max<int32_t>(nbc, 1));
      pack_offsets_units(al, *A, ta, oa, P.a_poff.p, P.a_base.p, s);
      OpIndex bu;
      make_op(ctx, B, !tb, bu);
      pack_offsets_units(al, *B, !tb, bu, P.b_poff.p, P.b_base.p, s);
    } else {      // FP64 k-pair slabs
      pack_offsets(al, *A, ta, P.a_poff.p, s);
      pack_offsets(al, *B, !tb, P.b_poff.p, s);
    }
  }
  DBuf<int4> bent(al, (size_t)std::max<int64_t>(ob.nnzb, 1));
  if (!fuse) product_records(ob, filt ? nb.p : nullptr, quads ? P.b_poff.p : nullptr, P.b_base.p, bent.p, s);
  // ------------------------------------------------------- a2: symbolic
  SymArgs sym;
  sym.a = &oa;
  sym.b = &ob;
  sym.nbc = nbc;
  // rows in the planner's locality order: neighbouring rows share most of
  // their op(B) rows, so the row-parallel kernels reuse them through L2
  sym.ord = nbr > 0 ? row_order(ctx, A) : nullptr;
  sym.retain = retain != 0;
  sym.use_cold = (beta != 0.0) && !retain && C0;
  DBuf<uint32_t> sym_bits;
  if (!retain) {
    const size_t nw = symbolic_bits_words(nbr, nbc);
    if (nw > 0) {
      sym_bits = DBuf<uint32_t>(al, nw);
      sym.bits = sym_bits.p;
    }
  }
  if (C0) {
    sym.cold_rp = C0->d_row_ptr;
    sym.cold_ci = C0->d_col_idx;
  }
  P.c_rp = DBuf<int64_t>(al, (size_t)nbr + 1);
  int64_t nnzb_c = 0;
  int32_t max_row = 0;
  {
    DBuf<int64_t> row_nnz(al, std::max<int32_t>(nbr, 1));
    if (retain) {
      // pattern = C_old pattern; row lengths from its row_ptr
      HIPCHECK(hipMemcpyAsync(P.c_rp.p, C0->d_row_ptr, sizeof(int64_t) * ((size_t)nbr + 1), hipMemcpyDeviceToDevice, s));
      nnzb_c = C0->nnzb;
      // max row length on the host side from a read-back of row_ptr
      std::vector<int64_t> h(nbr + 1);
      HIPCHECK(hipMemcpyAsync(h.data(), C0->d_row_ptr, sizeof(int64_t) * ((size_t)nbr + 1), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (int32_t i = 0; i < nbr; i++) max_row = std::max<int32_t>(max_row, (int32_t)(h[i + 1] - h[i]));
    } else {
      symbolic_count(sym, row_nnz.p, nullptr, s);
      if (nbr > 0) {
        exclusive_scan_i64(al, row_nnz.p, P.c_rp.p, nbr, s);
      } else {
        HIPCHECK(hipMemsetAsync(P.c_rp.p, 0, sizeof(int64_t), s));
      }
      PlanTotals T;
      T.at[0] = P.c_rp.p + nbr;
      if (fuse) {   // packed sizes, for the fused packing below
        T.at[1] = P.a_poff.p + A->nnzb;
        T.at[2] = P.b_poff.p + B->nnzb;
      }
      T.mx64 = row_nnz.p;   // widest result row
      T.nmx = nbr;
      DBuf<int64_t> tot(al, 8);
      plan_totals(T, tot.p, s);
      HIPCHECK(hipMemcpyAsync(ctx->pinned, tot.p, sizeof(int64_t) * 8, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      if (fuse) {
        P.a_pack_n = ctx->pinned[1];
        P.b_pack_n = ctx->pinned[2];
        P.a_pack = DBuf<double>(al, (size_t)std::max<int64_t>(P.a_pack_n, 2));
        P.b_pack = DBuf<double>(al, (size_t)std::max<int64_t>(P.b_pack_n, 2));
        pack_values(*A, ta, P.a_poff.p, P.a_pack.p, *B, !tb, P.b_poff.p, P.b_pack.p, s, na.p, nb.p);
        P.packed = true;
        product_records(ob, nb.p, P.b_poff.p, P.b_base.p, bent.p, s);
      }
      nnzb_c = ctx->pinned[0];
      max_row = (int32_t)ctx->pinned[7];
    }
  }
  P.nnzb_c = nnzb_c;
  if (nnzb_c > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "more than 2^31 result blocks");
  if (A->nnzb > INT32_MAX || B->nnzb > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "more than 2^31 operand blocks");
  const size_t nc1 = (size_t)std::max<int64_t>(nnzb_c, 1);
  // budget of the result pattern's phase, checked before any of its launches:
  // C's index and offsets, per-block counters and run starts, per-row sums
  {
    const size_t nks = quads ? ksizes.size() : 1;
    al.check(nc1 * (4 + 4 + 4 + 8 + 8 + 8 + 8 * nks) + 32 * ((size_t)nbr + 1) + 4096, "the result pattern");
  }
  P.c_ci = DBuf<int32_t>(al, nc1);
  P.c_row = DBuf<int32_t>(al, nc1);
  DBuf<int32_t> c_cnt(al, nc1);
  DBuf<int64_t> c_size(al, nc1), row_kmn(al, std::max<int32_t>(nbr, 1)), row_cand(al, std::max<int32_t>(nbr, 1)),
      row_real(al, std::max<int32_t>(nbr, 1));
  DBuf<int32_t> cnt_g;
  if (quads && (int64_t)max_row * (int64_t)ksizes.size() > SYM_CNT_CAP) {
    cnt_g = DBuf<int32_t>(al, nc1 * ksizes.size());
    HIPCHECK(hipMemsetAsync(cnt_g.p, 0, sizeof(int32_t) * nc1 * ksizes.size(), s));
  }
  HIPCHECK(hipMemsetAsync(c_cnt.p, 0, sizeof(int32_t) * nc1, s));
  // start of every k-size run inside its segment (quad path)
  DBuf<int32_t> kofs;
  if (quads) kofs = DBuf<int32_t>(al, nc1 * ksizes.size());
  FillArgs fa;
  fa.sym = sym;
  fa.c_rp = P.c_rp.p;
  fa.c_ci = P.c_ci.p;
  fa.c_row = P.c_row.p;
  fa.c_size = c_size.p;
  fa.c_cnt = c_cnt.p;
  fa.c_kflops = row_kmn.p;
  fa.row_cand = row_cand.p;
  fa.row_real = row_real.p;
  fa.pad4 = quads;
  fa.ksizes = ksizes;
  fa.cnt_g = cnt_g.p;
  fa.kofs = kofs.p;
  if (lowp && !quads && nnzb_c > 0)
    fail(BSMM_ERR_UNSUPPORTED, "FP32 / split modes need packed operands below 2 GB and at most 8 distinct k block sizes");
  // the diagonal-packed GEMM variant (blocks with both edges <= 8) takes
  // its products in groups of eight: such runs are padded to eight
  const bool diag8 = quads && !lowp && ctx->gemm_variant[0] == 3;
  fa.diag8 = diag8;
  fa.na = filt ? na.p : nullptr;
  fa.bent = bent.p;
  fa.eps = eps;
  fa.max_row = max_row;
  if (filt && !P.one_shot) {   // a plan records what its filter decisions rest on
    P.margin = DBuf<double>(al, 2);
    set_pairs(P.margin.p, 2, INFINITY, 0.0, s);
    fa.margin = P.margin.p;
  }
  symbolic_fill(fa, s);
  // column windows of the stack generator (bounds of C's and op(B)'s rows)
  const StackWindows sw = stack_windows(nbc, max_row, quads ? (int)ksizes.size() : 1);
  DBuf<int64_t> wslot, bwin;
  DBuf<int32_t> dmax_ns;
  if (sw.nwin > 0 && nnzb_c > 0) {
    wslot = DBuf<int64_t>(al, (size_t)nbr * (sw.nwin + 1));
    bwin = DBuf<int64_t>(al, (size_t)std::max<int32_t>(ob.nbr, 1) * (sw.nwin + 1));
    dmax_ns = DBuf<int32_t>(al, (size_t)std::max<int32_t>(nbr, 1));   // per row
    window_bounds(P.c_rp.p, P.c_ci.p, nbr, sw, wslot.p, dmax_ns.p, s);
    window_bounds(ob.row_ptr, ob.col_idx, ob.nbr, sw, bwin.p, nullptr, s);
  }
  P.c_off = DBuf<int64_t>(al, nc1 + 1);
  P.seg_off = DBuf<int64_t>(al, nc1 + 1);
  exclusive_scan_i64(al, c_size.p, P.c_off.p, nnzb_c, s);
  exclusive_scan_i32(al, c_cnt.p, P.seg_off.p, nnzb_c, s);
  // every size the rest of the plan needs, in one read-back
  {
    PlanTotals T;
    T.at[0] = P.c_off.p + nnzb_c;     // C values
    T.at[1] = P.seg_off.p + nnzb_c;   // stack entries, padding included
    if (quads) {
      T.at[2] = P.a_poff.p + A->nnzb;   // packed copies, in units of 8 bytes
      T.at[3] = P.b_poff.p + B->nnzb;
    }
    T.sum[0] = row_kmn.p;
    T.sum[1] = row_cand.p;
    T.sum[2] = row_real.p;
    T.n = nbr;
    if (sw.nwin > 0 && nnzb_c > 0) {   // most C blocks of one row in one window
      T.mx32 = dmax_ns.p;
      T.nmx = nbr;
    }
    DBuf<int64_t> tot(al, 8);
    plan_totals(T, tot.p, s);
    HIPCHECK(hipMemcpyAsync(ctx->pinned, tot.p, sizeof(int64_t) * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  P.nval_c = ctx->pinned[0];
  P.nstack = ctx->pinned[1];
  P.a_pack_n = quads ? ctx->pinned[2] : 0;
  P.b_pack_n = quads ? ctx->pinned[3] : 0;
  P.kmn_total = ctx->pinned[4];
  P.ncand = ctx->pinned[5];
  P.nprod = ctx->pinned[6];
  const int32_t max_ns = (int32_t)ctx->pinned[7];
  if (C0 && beta != 0.0 && nnzb_c > 0) {
    P.old_blk = DBuf<int32_t>(al, nc1);
    HIPCHECK(hipMemsetAsync(P.old_blk.p, 0xff, sizeof(int32_t) * nc1, s));
    old_block_map(C0->d_row_ptr, C0->d_col_idx, nbr, P.c_rp.p, P.c_ci.p, P.old_blk.p, s);
  }
  tm.mark();  // 3
  // budget of the stacks, the work list and (one-shot) the numeric buffers,
  // checked before any of their launches
  {
    size_t need = 8 * (size_t)std::max<int64_t>(P.nstack, 1) + nc1 * (4 + 4 + 4 + 32 + (units ? 16 : 0)) + 4096;
    if (P.one_shot)
      need += 8 * (size_t)std::max<int64_t>(P.nval_c, 1) + 8 * nc1 +
              (quads ? 8 * (size_t)(std::max<int64_t>(P.a_pack_n, 2) + std::max<int64_t>(P.b_pack_n, 2)) : 0);
    al.check(need, "the stacks and the numeric part");
  }
  // ------------------------------------------------------- a4: stacks
  P.stack = DBuf<int2>(al, (size_t)std::max<int64_t>(P.nstack, 1));
  {
    // rows wider than the stack generator's LDS cursors use global cursors,
    // one per (C block, k-size run)
    DBuf<int32_t> run;
    if (max_row > 4096 && !(sw.nwin > 0 && max_ns > 0)) {
      const size_t nr = nc1 * (quads ? ksizes.size() : 1);
      run = DBuf<int32_t>(al, nr);
      HIPCHECK(hipMemsetAsync(run.p, 0, sizeof(int32_t) * nr, s));
    }
    StackArgs sa;
    sa.a = &oa;
    sa.b = &ob;
    sa.c_rp = P.c_rp.p;
    sa.c_ci = P.c_ci.p;
    sa.seg_off = P.seg_off.p;
    sa.stack = P.stack.p;
    sa.na = filt ? na.p : nullptr;
    sa.eps = eps;
    sa.nbc = nbc;
    sa.nbr = nbr;
    sa.max_row = max_row;
    sa.ksizes = ksizes;
    sa.pad4 = quads;
    sa.encode = quads;
    sa.kofs = kofs.p;
    sa.a_poff = P.a_poff.p;
    sa.a_base = P.a_base.p;
    sa.bent = bent.p;
    sa.ord = sym.ord;
    sa.diag8 = diag8;
    if (sw.nwin > 0 && max_ns > 0) {
      sa.win = sw;
      sa.wslot = wslot.p;
      sa.bwin = bwin.p;
      sa.max_ns = max_ns;
    }
    if (P.nprod > 0) stack_fill(sa, run.p, s);
  }
  // GEMM work list: tiles of rows in the planner's locality order, columns
  // inside a tile in the same order when C is square over the same blocks.
  // A tile holds as many rows (16 to 256, at most nbr/16) as keep its rows
  // of op(A) within about 16 MB: 128 rows of 5/13 blocks took the GEMM of a
  // 4,000-row product from 11.37 to 10.97 ms against 16, while rows of
  // 23x23 blocks, five times the bytes, lost with tiles that tall.  Sorted
  // through per-subtile histograms while the key count stays modest; else
  // 16-row tiles, one workgroup each.
  DBuf<int32_t> wl_pos;   // place of every C block in the work list (sorted path)
  if (tiles && nnzb_c > 0) {
    // tiles of the result pattern and their step records; the per-block
    // stacks are not needed once merged into the steps
    const int32_t *ord = sym.ord;
    const int32_t *crank = (ord && nbc == nbr) ? ord + nbr : nullptr;
    OpRows ar;
    ar.rp = oa.row_ptr;
    ar.ci = oa.col_idx;
    ar.blk = oa.blk;
    ar.nnzb = oa.nnzb;
    OffsetAreas ob;
    ob.a_area = one_block_area(A);
    ob.b_area = one_block_area(B);
    ob.a_n = A->nnzb;
    ob.b_n = B->nnzb;
    build_tile_plan(al, TileShape{ctx->tile_ti, ctx->tile_tj}, ord, crank, crank ? ord : nullptr, nbr, nbc, P.c_rp.p,
                    P.c_ci.p, P.seg_off.p, P.stack.p, ar, (int32_t)opa_c.size(), oa.cbs, A->d_blk_off, B->d_blk_off,
                    ob, ctx->pinned, P.tp, s);
    P.stack.reset();
  } else if (nnzb_c > 0) {
    const int32_t *ord = row_order(ctx, A);
    DBuf<int32_t> seq;
    if (!ord && nbr >= 64 && nbr != A->nbc) {
      // no locality order of a rectangular A (a panel of rows): its rows in
      // index order, which the caller's numbering makes local (neighbouring
      // rows share most of their op(B) rows, so a tile's C blocks of one
      // column share their B blocks while those are in L2)
      seq = DBuf<int32_t>(al, (size_t)nbr);
      fill_sequence(seq.p, nbr, s);
      ord = seq.p;
    }
    if (ord) {
      P.c_list = DBuf<int32_t>(al, nc1);
      // columns in the locality order too when C is square over the same
      // blocks (row_order's second half: the rank of every row)
      const int32_t *rank = (nbc == nbr && !seq.p) ? ord + nbr : nullptr;
      const double row_bytes = 8.0 * (double)A->n_values / (double)std::max(nbr, 1);
      int32_t big = 16;
      while (big * 2 <= std::min(256, nbr / 16) && 2.0 * big * row_bytes <= 16.0 * (1 << 20)) big *= 2;
      const int64_t nkeys = (int64_t)((nbr + big - 1) / big) * nbc * (big / 16);
      const int32_t tile_rows = 16;
      if ((size_t)nbc * 4 <= 160 * 1024 && nkeys <= ((int64_t)1 << 24)) {
        if (quads) wl_pos = DBuf<int32_t>(al, nc1);
        build_work_list_sorted(al, ord, rank, P.c_rp.p, P.c_ci.p, nnzb_c, nbr, nbc, big, P.c_list.p, wl_pos.p, s);
      } else if ((size_t)nbc * 4 > 160 * 1024) {
        // columns too many for one LDS histogram: plain row order
        build_work_list(al, ord, nullptr, P.c_rp.p, P.c_ci.p, nbr, 0, tile_rows, P.c_list.p, s);
      } else {
        build_work_list(al, ord, rank, P.c_rp.p, P.c_ci.p, nbr, nbc, tile_rows, P.c_list.p, s);
      }
    }
  }
  // work-item descriptors of the quad path
  if (quads && nnzb_c > 0) {
    P.desc = DBuf<BlkDesc>(al, nc1);
    if (units) P.ubase = DBuf<UnitBases>(al, nc1);
    const DescBases bases{P.a_base.p, P.b_base.p, P.ubase.p};
    if (wl_pos.p)   // C blocks read in storage order, records written at their places
      build_desc_by_block(nnzb_c, wl_pos.p, P.c_row.p, P.c_ci.p, oa.rbs, ob.cbs, P.seg_off.p, P.c_off.p, bases,
                          P.desc.p, s);
    else
      build_desc(nnzb_c, P.c_list.p, P.c_row.p, P.c_ci.p, oa.rbs, ob.cbs, P.seg_off.p, P.c_off.p, bases, P.desc.p,
                 s);
  }
  if (filt && !P.one_shot) {
    P.na_plan = std::move(na);
    P.nb_plan = std::move(nb);
  }
  // ------------------------------------- buffers of the numeric part
  P.post = filt && !retain;
  {
    Plan::Ws &w = P.ws;
    size_t at = 0;
    auto region = [&](size_t bytes) {
      const size_t o = at;
      at += (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
      return o;
    };
    if (quads && P.nprod > 0) {   // packed copies (sizes in units of 8 bytes)
      w.has_apack = true;
      w.apack = region(8 * (size_t)std::max<int64_t>(P.a_pack_n, 2));
      w.bpack = region(8 * (size_t)std::max<int64_t>(P.b_pack_n, 2));
      if (ctx->mode == BSMM_COMPUTE_SPLIT) {
        w.has_alo = true;
        w.alo = region(8 * (size_t)std::max<int64_t>(P.a_pack_n, 2));
        w.blo = region(8 * (size_t)std::max<int64_t>(P.b_pack_n, 2));
      }
    }
    if (!quads && !tiles && ta && P.nprod > 0) {
      w.has_at = true;
      w.at = region(8 * (size_t)std::max<int64_t>(A->n_values, 1));
    }
    if (!quads && !tiles && !tb && P.nprod > 0) {
      w.has_bt = true;
      w.bt = region(8 * (size_t)std::max<int64_t>(B->n_values, 1));
    }
    if (P.post) {
      w.has_cnorm = true;
      w.cnorm = region(8 * nc1);
    }
    w.core = at;
    if (P.post) w.stash = region(8 * (size_t)std::max<int64_t>(P.nval_c, 1));
    w.total = at;
  }
  if (P.one_shot) {   // the one-shot product's buffers come from the library (C values become the result)
    if (P.packed) {   // fused packing already wrote the packed copies
      P.c_values = DBuf<double>(al, (size_t)std::max<int64_t>(P.nval_c, 1));
      if (P.post) P.c_norm = DBuf<double>(al, nc1);
    } else {
      P.c_values = DBuf<double>(al, (size_t)std::max<int64_t>(P.nval_c, 1));
      P.own_ws = DBuf<uint8_t>(al, std::max<size_t>(P.ws.core, 256));
    }
  }
  if (!ctx->zeros) {
    ctx->zeros = static_cast<double *>(al.alloc(4096));
    HIPCHECK(hipMemsetAsync(ctx->zeros, 0, 4096, s));
  }
  GemmArgs &ga = P.ga;
  ga.a = &oa;
  ga.b = &ob;
  ga.c_list = P.c_list.p;
  ga.desc = P.desc.p;
  ga.ubase = P.ubase.p;
  ga.c_row = P.c_row.p;
  ga.c_ci = P.c_ci.p;
  ga.c_off = P.c_off.p;
  ga.seg_off = P.seg_off.p;
  ga.stack = P.stack.p;
  ga.c_old_blk = P.old_blk.p;
  ga.old_off = C0 ? C0->d_blk_off : nullptr;
  ga.old_values = C0 ? C0->d_values : nullptr;
  ga.alpha = P.alpha;
  ga.beta = P.beta;
  ga.mode = ctx->mode;
  ga.a_bytes = (uint64_t)(quads ? P.a_pack_n : A->n_values) * sizeof(double);
  ga.b_bytes = (uint64_t)(quads ? P.b_pack_n : B->n_values) * sizeof(double);
  ga.zeros = ctx->zeros;
  ga.quads = quads;
  for (int t = 0; t < 16; t++) ga.variant[t] = ctx->gemm_variant[t];
  TileArgs &tg = P.targs;
  tg.rbs = oa.rbs;
  tg.cbs = ob.cbs;
  tg.a_val = A->d_values;
  tg.b_val = B->d_values;
  tg.a_n = A->n_values;
  tg.b_n = B->n_values;
  tg.ta = ta;
  tg.tb = tb;
  tg.c_off = P.c_off.p;
  tg.old_blk = P.old_blk.p;
  tg.old_off = C0 ? C0->d_blk_off : nullptr;
  tg.old_val = C0 ? C0->d_values : nullptr;
  tg.alpha = P.alpha;
  tg.beta = P.beta;
  tg.uni = P.uni;
  tg.xcd_chunk = ctx->tile_chunk;
  P.max_edge = 1;
  for (int32_t v : opa_r) P.max_edge = std::max(P.max_edge, v);
  for (int32_t v : opb_c) P.max_edge = std::max(P.max_edge, v);
  if (P.one_shot) {
    if (P.packed) bind_packed(P);
    else bind_numeric(P, P.c_values.p, P.own_ws.p);
  }
  tm.mark();  // 4
}

// The numeric part: operand copies and the block GEMM (kernels only).
static void plan_numeric(Plan &P, bool marks) {
  hipStream_t s = P.ctx->stream;
  const bool ta = P.ta, tb = P.tb;
  if (P.tiles) {   // operands come straight from the stored values
    if (marks) P.tm.mark();  // 5
    tile_gemm_launch(P.tp, P.targs, s);
    if (marks) P.tm.mark();  // 6
    return;
  }
  if (P.nprod > 0) {
    GemmArgs &ga = P.ga;
    if (P.quads && P.lowp) {
      pack32_values(*P.A, ta, P.a_poff.p, const_cast<float *>(ga.a_hi), const_cast<float *>(ga.a_lo), s);
      pack32_values(*P.B, !tb, P.b_poff.p, const_cast<float *>(ga.b_hi), const_cast<float *>(ga.b_lo), s);
    } else if (P.quads) {
      if (!P.packed)
        pack_values(*P.A, ta, P.a_poff.p, const_cast<double *>(ga.a_pack), *P.B, !tb, P.b_poff.p,
                    const_cast<double *>(ga.b_pack), s);
      P.packed = false;   // a later execution packs the values it finds
    } else {
      if (ta) transpose_blocks(*P.A, const_cast<double *>(ga.a_cm), s);
      if (!tb) transpose_blocks(*P.B, const_cast<double *>(ga.b_rm), s);
    }
  }
  if (marks) P.tm.mark();  // 5
  if (P.lowp)
    gemm_launch_lowp(P.ga, P.nnzb_c, P.max_edge, s);
  else
    gemm_launch(P.ga, P.nnzb_c, P.max_edge, s);
  if (marks) P.tm.mark();  // 6
}

// Post-filter and the result matrix.  consume: the plan's C buffers become
// the result (one-shot multiply); otherwise they are copied.
static bsmm_mat_s *plan_finish(Plan &P, bool consume) {
  bsmm_ctx ctx = P.ctx;
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  const int64_t nnzb_c = P.nnzb_c;
  bsmm_mat_s *R = new_result(ctx, P.nbr, P.nbc, P.opa_r, P.opb_c);
  try {
    int64_t kept = nnzb_c;
    DBuf<int64_t> rank;
    if (P.post && nnzb_c > 0) {
      CompactArgs ca;
      ca.nbr = P.nbr;
      ca.nnzb = nnzb_c;
      ca.rp = P.c_rp.p;
      ca.ci = P.c_ci.p;
      ca.off = P.c_off.p;
      ca.values = P.cval;
      ca.norm = P.ga.c_norm;
      ca.eps = P.eps;
      DBuf<int32_t> flags(al, (size_t)std::max<int64_t>(nnzb_c, 1));
      kept = count_kept(al, ca, flags.p, ctx->pinned, s, rank);
      if (kept < nnzb_c) {
        DBuf<int64_t> nrp(al, (size_t)P.nbr + 1), noff(al, (size_t)std::max<int64_t>(kept, 1) + 1);
        DBuf<int32_t> nci(al, (size_t)std::max<int64_t>(kept, 1));
        double *nv = nullptr;
        int64_t nval = 0;
        compact(al, ca, rank.p, P.oa.rbs, P.ob.cbs, nrp.p, nci.p, noff.p, ctx->pinned, &nv, &nval, s);
        R->d_row_ptr = nrp.release_ownership();
        R->d_col_idx = nci.release_ownership();
        R->d_blk_off = noff.release_ownership();
        R->d_values = nv;
        R->nnzb = kept;
        R->n_values = nval;
      }
    }
    if (kept == nnzb_c) {
      if (consume) {
        R->d_row_ptr = P.c_rp.release_ownership();
        R->d_col_idx = P.c_ci.release_ownership();
        R->d_blk_off = P.c_off.release_ownership();
        R->d_values = P.c_values.release_ownership();
      } else {
        const size_t nc1 = (size_t)std::max<int64_t>(nnzb_c, 1);
        R->d_row_ptr = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)P.nbr + 1)));
        R->d_col_idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nc1));
        R->d_blk_off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * (nc1 + 1)));
        R->d_values = static_cast<double *>(al.alloc(sizeof(double) * (size_t)std::max<int64_t>(P.nval_c, 1)));
        HIPCHECK(hipMemcpyAsync(R->d_row_ptr, P.c_rp.p, sizeof(int64_t) * ((size_t)P.nbr + 1), hipMemcpyDeviceToDevice, s));
        if (nnzb_c) {
          HIPCHECK(hipMemcpyAsync(R->d_col_idx, P.c_ci.p, sizeof(int32_t) * (size_t)nnzb_c, hipMemcpyDeviceToDevice, s));
          HIPCHECK(hipMemcpyAsync(R->d_values, P.cval, sizeof(double) * (size_t)P.nval_c, hipMemcpyDeviceToDevice, s));
        }
        HIPCHECK(hipMemcpyAsync(R->d_blk_off, P.c_off.p, sizeof(int64_t) * ((size_t)nnzb_c + 1), hipMemcpyDeviceToDevice, s));
      }
      R->nnzb = nnzb_c;
      R->n_values = P.nval_c;
    }
  } catch (...) {
    free_mat(R);
    throw;
  }
  return R;
}

static int32_t gemm_path(const Plan &P) {
  return P.tiles ? (P.uni ? 4 : 2) : P.lowp ? 3 : P.quads ? (P.units ? 5 : 0) : 1;
}

// Post-filter and the result matrix of an execution into caller buffers:
// the result's index belongs to the library, its values are the caller's
// (borrowed).  When the post-filter drops blocks, the values are copied to
// the workspace's stash and compacted back into the caller's buffer.
static bsmm_mat_s *plan_finish_into(Plan &P) {
  bsmm_ctx ctx = P.ctx;
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  const int64_t nnzb_c = P.nnzb_c;
  bsmm_mat_s *R = new_result(ctx, P.nbr, P.nbc, P.opa_r, P.opb_c);
  R->owns_values = false;
  try {
    int64_t kept = nnzb_c;
    if (P.post && nnzb_c > 0) {
      CompactArgs ca;
      ca.nbr = P.nbr;
      ca.nnzb = nnzb_c;
      ca.rp = P.c_rp.p;
      ca.ci = P.c_ci.p;
      ca.off = P.c_off.p;
      ca.values = P.cval;
      ca.norm = P.ga.c_norm;
      ca.eps = P.eps;
      DBuf<int32_t> flags(al, (size_t)std::max<int64_t>(nnzb_c, 1));
      DBuf<int64_t> rank;
      kept = count_kept(al, ca, flags.p, ctx->pinned, s, rank);
      if (kept < nnzb_c) {
        double *stash = reinterpret_cast<double *>(P.wsp + P.ws.stash);
        HIPCHECK(hipMemcpyAsync(stash, P.cval, sizeof(double) * (size_t)P.nval_c, hipMemcpyDeviceToDevice, s));
        ca.values = stash;
        DBuf<int64_t> nrp(al, (size_t)P.nbr + 1), noff(al, (size_t)std::max<int64_t>(kept, 1) + 1);
        DBuf<int32_t> nci(al, (size_t)std::max<int64_t>(kept, 1));
        double *nv = P.cval;
        int64_t nval = 0;
        compact(al, ca, rank.p, P.oa.rbs, P.ob.cbs, nrp.p, nci.p, noff.p, ctx->pinned, &nv, &nval, s, P.cval);
        R->d_row_ptr = nrp.release_ownership();
        R->d_col_idx = nci.release_ownership();
        R->d_blk_off = noff.release_ownership();
        R->d_values = P.cval;
        R->nnzb = kept;
        R->n_values = nval;
      }
    }
    if (kept == nnzb_c) {
      const size_t nc1 = (size_t)std::max<int64_t>(nnzb_c, 1);
      R->d_row_ptr = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)P.nbr + 1)));
      R->d_col_idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nc1));
      R->d_blk_off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * (nc1 + 1)));
      HIPCHECK(hipMemcpyAsync(R->d_row_ptr, P.c_rp.p, sizeof(int64_t) * ((size_t)P.nbr + 1), hipMemcpyDeviceToDevice, s));
      if (nnzb_c)
        HIPCHECK(hipMemcpyAsync(R->d_col_idx, P.c_ci.p, sizeof(int32_t) * (size_t)nnzb_c, hipMemcpyDeviceToDevice, s));
      HIPCHECK(hipMemcpyAsync(R->d_blk_off, P.c_off.p, sizeof(int64_t) * ((size_t)nnzb_c + 1), hipMemcpyDeviceToDevice, s));
      R->d_values = P.cval;
      R->nnzb = nnzb_c;
      R->n_values = P.nval_c;
    }
  } catch (...) {
    free_mat(R);
    throw;
  }
  return R;
}

static void plan_info(Plan &P, const bsmm_mat_s *R, bsmm_multiply_info *info) {
  if (!info) return;
  Timer &tm = P.tm;
  info->c_nnzb_symbolic = P.nnzb_c;
  info->c_nnzb = R ? R->nnzb : P.nnzb_c;
  info->c_n_values = R ? R->n_values : P.nval_c;
  info->n_products = P.nprod;
  info->n_candidates = P.ncand;
  info->useful_flops = 2.0 * (double)P.kmn_total;
  info->ms_index = tm.between(0, 1);
  info->ms_norms = tm.between(1, 2);
  info->ms_symbolic = tm.between(2, 3);
  info->ms_stacks = tm.between(3, 4) + tm.between(4, 5);   // stacks, work list, operand copies
  info->ms_gemm = tm.between(5, 6);
  info->ms_filter = tm.between(6, 7);
  info->ms_total = tm.between(0, 7);
  info->gemm_path = gemm_path(P);
}

static bsmm_mat_s *multiply_impl(bsmm_ctx ctx, char transa, char transb, double alpha, bsmm_mat_s *A,
                                 bsmm_mat_s *B, double beta, bsmm_mat_s *C0, double eps, int retain,
                                 bsmm_multiply_info *info) {
  Plan P(ctx);
  P.A = A;
  P.B = B;
  P.C0 = C0;
  P.alpha = alpha;
  P.beta = beta;
  P.eps = eps;
  P.retain = retain;
  P.one_shot = true;
  plan_build(P, transa, transb);
  plan_numeric(P, true);
  bsmm_mat_s *R = plan_finish(P, true);
  P.tm.mark();  // 7
  try {
    plan_info(P, R, info);
  } catch (...) {
    free_mat(R);
    throw;
  }
  return R;
}

// Deep copy of a matrix (owned index and values), ordered on the stream.
static bsmm_mat_s *copy_matrix(bsmm_ctx ctx, const bsmm_mat_s *x) {
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  bsmm_mat_s *m = new_result(ctx, x->nbr, x->nbc, x->h_rbs, x->h_cbs);
  try {
    const size_t nb1 = (size_t)std::max<int64_t>(x->nnzb, 1);
    m->d_row_ptr = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)x->nbr + 1)));
    m->d_col_idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * nb1));
    m->d_blk_off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * (nb1 + 1)));
    m->d_values = static_cast<double *>(al.alloc(sizeof(double) * (size_t)std::max<int64_t>(x->n_values, 1)));
    m->nnzb = x->nnzb;
    m->n_values = x->n_values;
    HIPCHECK(hipMemcpyAsync(m->d_row_ptr, x->d_row_ptr, sizeof(int64_t) * ((size_t)x->nbr + 1),
                            hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(m->d_blk_off, x->d_blk_off, sizeof(int64_t) * ((size_t)x->nnzb + 1),
                            hipMemcpyDeviceToDevice, s));
    if (x->nnzb)
      HIPCHECK(hipMemcpyAsync(m->d_col_idx, x->d_col_idx, sizeof(int32_t) * (size_t)x->nnzb, hipMemcpyDeviceToDevice, s));
    if (x->n_values)
      HIPCHECK(hipMemcpyAsync(m->d_values, x->d_values, sizeof(double) * (size_t)x->n_values, hipMemcpyDeviceToDevice, s));
  } catch (...) {
    free_mat(m);
    throw;
  }
  return m;
}

// Whether x and y have the same block sizes and block pattern (one
// synchronisation when the sizes agree).
static bool same_pattern(bsmm_ctx ctx, const bsmm_mat_s *x, const bsmm_mat_s *y) {
  if (x == y) return true;
  if (x->nbr != y->nbr || x->nbc != y->nbc || x->nnzb != y->nnzb || x->h_rbs != y->h_rbs || x->h_cbs != y->h_cbs)
    return false;
  hipStream_t s = ctx->stream;
  DBuf<int32_t> flag(ctx->alloc, 1);
  HIPCHECK(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
  differs_i64(x->d_row_ptr, y->d_row_ptr, (int64_t)x->nbr + 1, flag.p, s);
  differs_i32(x->d_col_idx, y->d_col_idx, x->nnzb, flag.p, s);
  HIPCHECK(hipMemcpyAsync(ctx->pinned, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return *reinterpret_cast<int32_t *>(ctx->pinned) == 0;
}

// Whether every on-the-fly filter decision of plan P stays the same when its
// operands take the values of A and B (same patterns as the plan's).  First
// a bound: each norm product of the plan moves by a factor within
// [fa_lo fb_lo, fa_hi fb_hi] (the ranges of the per-block norm ratios now /
// then); the decisions hold when the smallest kept product stays >= eps and
// the largest dropped one stays < eps under those factors, with a relative
// slack of 1e-12 for the rounding of the products.  When the bound is
// inconclusive, every candidate's decision is recomputed under both sets of
// norms and compared exactly.
static bool filter_decisions_hold(Plan &P, const bsmm_mat_s *A, const bsmm_mat_s *B) {
  if (!P.filt) return true;
  bsmm_ctx ctx = P.ctx;
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  DBuf<double> na(al, (size_t)std::max<int64_t>(A->nnzb, 1)), nb(al, (size_t)std::max<int64_t>(B->nnzb, 1));
  DBuf<double> rb(al, 4);
  set_pairs(rb.p, 4, INFINITY, 0.0, s);
  block_norms(*A, na.p, s);
  ratio_bounds(P.na_plan.p, na.p, A->nnzb, rb.p, s);
  block_norms(*B, nb.p, s);
  ratio_bounds(P.nb_plan.p, nb.p, B->nnzb, rb.p + 2, s);
  double h[6];
  HIPCHECK(hipMemcpyAsync(ctx->pinned, rb.p, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(ctx->pinned + 4, P.margin.p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  std::memcpy(h, ctx->pinned, sizeof h);
  const double fa_lo = h[0], fa_hi = h[1], fb_lo = h[2], fb_hi = h[3], kept_min = h[4], drop_max = h[5];
  const double eps = P.eps, slack = 1e-12;
  const bool kept_ok = kept_min == INFINITY || kept_min * fa_lo * fb_lo >= eps * (1.0 + slack);
  const bool drop_ok = drop_max == 0.0 || drop_max * fa_hi * fb_hi <= eps * (1.0 - slack);
  if (kept_ok && drop_ok && fa_hi < INFINITY && fb_hi < INFINITY) return true;
  // the bound is inconclusive: decide every candidate product under both
  // sets of norms and compare (a pass over the candidates, no stacks)
  DBuf<int32_t> flag(al, 1);
  HIPCHECK(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
  decisions_differ(P.oa, P.ob, P.na_plan.p, P.nb_plan.p, na.p, nb.p, eps, flag.p, s);
  HIPCHECK(hipMemcpyAsync(ctx->pinned, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return *reinterpret_cast<int32_t *>(ctx->pinned) == 0;
}

// One multiplication of a loop whose operand patterns settle (the sign
// iteration): the plan of the previous call is re-executed on the new values
// when the patterns of A and B are those it was built on and its filter
// decisions provably stay the same; otherwise a new plan is built.  The plan
// reads deep copies of A and B held by the cache, so the caller may free its
// matrices; the result is a new matrix either way, equal to bsmm_multiply's.
struct MulCache {
  Plan *P = nullptr;
  bsmm_mat_s *a = nullptr, *b = nullptr;   // copies the plan reads (b == a for A == B)
  bool same = false;
  int32_t reuses = 0;
  void clear() {
    delete P;
    P = nullptr;
    if (b && b != a) free_mat(b);
    if (a) free_mat(a);
    a = b = nullptr;
  }
  ~MulCache() { clear(); }
};

static bsmm_mat_s *multiply_cached(bsmm_ctx ctx, MulCache &mc, double alpha, bsmm_mat_s *A, bsmm_mat_s *B,
                                   double beta, bsmm_mat_s *C0, double eps, bsmm_multiply_info *info) {
  hipStream_t s = ctx->stream;
  const bool same = A == B;
  bool reuse = mc.P && mc.same == same && same_pattern(ctx, A, mc.a) && (same || same_pattern(ctx, B, mc.b));
  if (reuse) reuse = filter_decisions_hold(*mc.P, A, B);
  if (reuse) {
    if (A != mc.a && A->n_values)
      HIPCHECK(hipMemcpyAsync(mc.a->d_values, A->d_values, sizeof(double) * (size_t)A->n_values,
                              hipMemcpyDeviceToDevice, s));
    if (!same && B != mc.b && B->n_values)
      HIPCHECK(hipMemcpyAsync(mc.b->d_values, B->d_values, sizeof(double) * (size_t)B->n_values,
                              hipMemcpyDeviceToDevice, s));
    mc.reuses++;
  } else {
    mc.clear();
    mc.a = copy_matrix(ctx, A);
    mc.b = same ? mc.a : copy_matrix(ctx, B);
    mc.same = same;
    mc.P = new Plan(ctx);
    Plan &P = *mc.P;
    P.A = mc.a;
    P.B = mc.b;
    P.C0 = C0;
    P.alpha = alpha;
    P.beta = beta;
    P.eps = eps;
    P.retain = 0;
    plan_build(P, 'N', 'N');
  }
  Plan &P = *mc.P;
  ensure_own_buffers(P);
  plan_numeric(P, false);
  bsmm_mat_s *R = plan_finish(P, false);
  if (info) {
    *info = bsmm_multiply_info{};
    info->c_nnzb_symbolic = P.nnzb_c;
    info->c_nnzb = R->nnzb;
    info->c_n_values = R->n_values;
    info->n_products = P.nprod;
    info->n_candidates = P.ncand;
    info->useful_flops = 2.0 * (double)P.kmn_total;
    info->gemm_path = gemm_path(P);
  }
  return R;
}

// Block-diagonal identity with the given block sizes (owned values).
static bsmm_mat_s *make_identity(bsmm_ctx ctx, const std::vector<int32_t> &sizes) {
  const int32_t n = (int32_t)sizes.size();
  bsmm_mat_s *I = new_result(ctx, n, n, sizes, sizes);
  Allocator &al = ctx->alloc;
  try {
    std::vector<int64_t> rp((size_t)n + 1), off((size_t)n + 1);
    std::vector<int32_t> ci((size_t)std::max(n, 1));
    off[0] = 0;
    for (int32_t i = 0; i < n; i++) {
      rp[i] = i;
      ci[i] = i;
      off[i + 1] = off[i] + (int64_t)sizes[i] * sizes[i];
    }
    rp[n] = n;
    I->nnzb = n;
    I->n_values = off[n];
    I->d_row_ptr = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)n + 1)));
    I->d_col_idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * (size_t)std::max(n, 1)));
    I->d_blk_off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)n + 1)));
    I->d_values = static_cast<double *>(al.alloc(sizeof(double) * (size_t)std::max<int64_t>(off[n], 1)));
    upload(I->d_row_ptr, rp.data(), sizeof(int64_t) * rp.size(), ctx->stream);
    upload(I->d_col_idx, ci.data(), sizeof(int32_t) * (size_t)n, ctx->stream);
    upload(I->d_blk_off, off.data(), sizeof(int64_t) * off.size(), ctx->stream);
    identity_values(I->d_rbs, I->d_blk_off, n, I->d_values, ctx->stream);
    HIPCHECK(hipStreamSynchronize(ctx->stream));   // host vectors go out of scope
  } catch (...) {
    free_mat(I);
    throw;
  }
  return I;
}

// ||X^2 - I||_F from T = 3I - X^2 (= ||T - 2I||_F), summed per block row.
static double sign_residual(bsmm_ctx ctx, const bsmm_mat_s &T) {
  Allocator &al = ctx->alloc;
  DBuf<double> rows(al, (size_t)std::max(T.nbr, 1));
  shift_dist_rows(T, 2.0, rows.p, ctx->stream);
  std::vector<double> h((size_t)T.nbr);
  if (T.nbr) HIPCHECK(hipMemcpyAsync(h.data(), rows.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  double ss = 0.0;
  for (double v : h) ss += v;   // fixed order: deterministic
  return std::sqrt(ss);
}

// Newton-Schulz sign iteration, X <- 1/2 X (3I - X^2): two filtered
// multiplications per iteration.
static bsmm_mat_s *sign_impl(bsmm_ctx ctx, bsmm_mat_s *X0, int32_t max_iter, double eps, double tol,
                             bsmm_sign_info *info, double *trace_res, int64_t *trace_nnzb) {
  if (X0->nbr != X0->nbc) fail(BSMM_ERR_SHAPE, "the sign iteration needs a square block grid");
  if (X0->h_rbs != X0->h_cbs) fail(BSMM_ERR_SHAPE, "row and column block sizes differ");
  if (max_iter < 0) fail(BSMM_ERR_INVALID_ARG, "max_iter < 0");
  if (!(eps >= 0.0)) fail(BSMM_ERR_INVALID_ARG, "filter_eps must be >= 0");
  double ndim = 0.0;
  for (int32_t v : X0->h_rbs) ndim += v;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipEventRecord(e0, ctx->stream));
  }
  bsmm_mat_s *I = make_identity(ctx, X0->h_rbs);
  bsmm_mat_s *X = X0;   // borrowed until the first update
  // plans of the two multiplications, re-executed while the patterns of X
  // and T stay put and the filter decisions provably do not change
  MulCache m1, m2;
  bsmm_sign_info st{};
  st.nnzb_max = X0->nnzb;
  st.residual = -1.0;
  try {
    for (int32_t it = 0; it < max_iter; it++) {
      bsmm_multiply_info mi{};
      // T = 3I - X X  (beta = 3, C_old = I: the pattern is the union)
      bsmm_mat_s *T = multiply_cached(ctx, m1, -1.0, X, X, 3.0, I, eps, &mi);
      st.useful_flops += mi.useful_flops;
      st.nnzb_max = std::max(st.nnzb_max, T->nnzb);
      double res;
      try {
        res = (ndim > 0 ? sign_residual(ctx, *T) / std::sqrt(ndim) : 0.0);
      } catch (...) {
        free_mat(T);
        throw;
      }
      st.residual = res;
      st.iterations = it + 1;
      if (trace_res) trace_res[it] = res;
      if (tol > 0.0 && res < tol) {
        free_mat(T);
        st.converged = 1;
        if (trace_nnzb) trace_nnzb[it] = X->nnzb;
        break;
      }
      bsmm_mat_s *Xn;
      try {
        Xn = multiply_cached(ctx, m2, 0.5, X, T, 0.0, nullptr, eps, &mi);
      } catch (...) {
        free_mat(T);
        throw;
      }
      st.useful_flops += mi.useful_flops;
      free_mat(T);
      if (X != X0) free_mat(X);
      X = Xn;
      st.nnzb_max = std::max(st.nnzb_max, X->nnzb);
      if (trace_nnzb) trace_nnzb[it] = X->nnzb;
    }
    if (X == X0) {   // no update ran: return a copy of X0's blocks
      bsmm_multiply_info mi{};
      X = multiply_impl(ctx, 'N', 'N', 1.0, X0, I, 0.0, nullptr, 0.0, 0, &mi);
    }
  } catch (...) {
    if (X != X0) free_mat(X);
    free_mat(I);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    throw;
  }
  st.plan_reuses = m1.reuses + m2.reuses;
  m1.clear();
  m2.clear();
  free_mat(I);
  st.nnzb = X->nnzb;
  if (ctx->timing) {
    HIPCHECK(hipEventRecord(e1, ctx->stream));
    HIPCHECK(hipEventSynchronize(e1));
    HIPCHECK(hipEventElapsedTime(&st.ms_total, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (info) *info = st;
  return X;
}

}  // namespace bsmm

using namespace bsmm;

extern "C" {

const char *bsmm_status_string(bsmm_status s) {
  switch (s) {
    case BSMM_OK: return "BSMM_OK";
    case BSMM_ERR_INVALID_ARG: return "BSMM_ERR_INVALID_ARG";
    case BSMM_ERR_BAD_INDEX: return "BSMM_ERR_BAD_INDEX";
    case BSMM_ERR_SHAPE: return "BSMM_ERR_SHAPE";
    case BSMM_ERR_ALIAS: return "BSMM_ERR_ALIAS";
    case BSMM_ERR_OUT_OF_MEMORY: return "BSMM_ERR_OUT_OF_MEMORY";
    case BSMM_ERR_DEVICE: return "BSMM_ERR_DEVICE";
    case BSMM_ERR_UNSUPPORTED: return "BSMM_ERR_UNSUPPORTED";
  }
  return "BSMM_ERR_UNKNOWN";
}

const char *bsmm_last_error(void) { return g_last_error.c_str(); }

bsmm_status bsmm_ctx_create(int device, void *stream, size_t hbm_budget_bytes, bsmm_ctx *out) {
  ABI_BEGIN
  if (!out) fail(BSMM_ERR_INVALID_ARG, "out is NULL");
  int n = 0;
  HIPCHECK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) fail(BSMM_ERR_INVALID_ARG, "no such device");
  DeviceGuard g(device);
  auto *c = new bsmm_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->alloc.init(device, hbm_budget_bytes);
  try {
    noalloc_init(device);   // device address of the allocation-free filter's scratch array
  } catch (...) {
    delete c;
    throw;
  }
  if (hipHostMalloc((void **)&c->pinned, 64 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
    fail(BSMM_ERR_OUT_OF_MEMORY, "pinned host buffer");
  }
  *out = c;
  ABI_END
}

bsmm_status bsmm_ctx_set_stream(bsmm_ctx ctx, void *stream) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(ctx->device);
  // work queued on the old stream must finish before buffers are reused on the new one
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  ctx->stream = static_cast<hipStream_t>(stream);
  ABI_END
}

bsmm_status bsmm_ctx_set_timing(bsmm_ctx ctx, int enable) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  ctx->timing = enable != 0;
  ABI_END
}

bsmm_status bsmm_ctx_set_compute_mode(bsmm_ctx ctx, bsmm_compute_mode mode) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (mode != BSMM_COMPUTE_FP64 && mode != BSMM_COMPUTE_FP32 && mode != BSMM_COMPUTE_SPLIT)
    fail(BSMM_ERR_INVALID_ARG, "unknown compute mode");
  ctx->mode = mode;
  ABI_END
}

bsmm_status bsmm_ctx_set_gemm_variant(bsmm_ctx ctx, int32_t m, int32_t n, int32_t variant) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (m < 1 || m > MAX_BLOCK || n < 1 || n > MAX_BLOCK) fail(BSMM_ERR_INVALID_ARG, "block edge outside 1..32");
  if (variant < 0 || variant > 6) fail(BSMM_ERR_INVALID_ARG, "variant must be 0, 1, 2, 3, 4, 5 or 6");
  if ((variant == 5 || variant == 6) && (m < 17 || n < 17 || m > 24 || n > 24))
    fail(BSMM_ERR_INVALID_ARG, "variants 5 and 6 need both block edges in 17..24");
  if (variant == 3 && (m > 8 || n > 8)) fail(BSMM_ERR_INVALID_ARG, "variant 3 needs both block edges <= 8");
  if (variant == 4 && (m < 9 || n < 9 || m > 24 || n > 24 || (m <= 16 && n <= 16)))
    fail(BSMM_ERR_INVALID_ARG, "variant 4 needs both block edges in 9..24 and one above 16");
  ctx->gemm_variant[((m + 7) / 8 - 1) * 4 + ((n + 7) / 8 - 1)] = (uint8_t)variant;
  ABI_END
}

bsmm_status bsmm_ctx_set_tile_shape(bsmm_ctx ctx, int32_t ti, int32_t tj) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (!tile_shape_valid(ti, tj)) fail(BSMM_ERR_INVALID_ARG, "tile shape must be 2x2, 2x4, 4x2, 4x4, 4x8 or 8x4");
  ctx->tile_ti = ti;
  ctx->tile_tj = tj;
  ABI_END
}

bsmm_status bsmm_ctx_set_tile_schedule(bsmm_ctx ctx, int32_t persistent, int64_t xcd_chunk) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (xcd_chunk < 0 || xcd_chunk > (1ll << 30)) fail(BSMM_ERR_INVALID_ARG, "xcd_chunk must be in 0..2^30");
  if (persistent != 0) fail(BSMM_ERR_UNSUPPORTED, "the persistent tile launch is disabled");
  ctx->tile_chunk = xcd_chunk;
  ABI_END
}

bsmm_status bsmm_ctx_set_packed_addressing(bsmm_ctx ctx, int32_t mode) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (mode != 0 && mode != 1) fail(BSMM_ERR_INVALID_ARG, "addressing mode must be 0 (automatic) or 1 (per unit)");
  ctx->pack_addr = mode;
  ABI_END
}

bsmm_status bsmm_ctx_set_row_order(bsmm_ctx ctx, int32_t mode) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (mode < 0 || mode > 2) fail(BSMM_ERR_INVALID_ARG, "row order mode must be 0 (automatic), 1 (always) or 2 (never)");
  ctx->row_order = mode;
  ABI_END
}

bsmm_status bsmm_ctx_memory(bsmm_ctx ctx, size_t *held, size_t *peak) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (held) *held = ctx->alloc.held();
  if (peak) *peak = ctx->alloc.peak();
  ABI_END
}

bsmm_status bsmm_ctx_trim(bsmm_ctx ctx) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(ctx->device);
  ctx->alloc.trim();
  ABI_END
}

bsmm_status bsmm_ctx_synchronize(bsmm_ctx ctx) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(ctx->device);
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  ABI_END
}

bsmm_status bsmm_ctx_destroy(bsmm_ctx ctx) {
  ABI_BEGIN
  if (!ctx) fail(BSMM_ERR_INVALID_ARG, "ctx is NULL");
  if (ctx->live_mats != 0) fail(BSMM_ERR_INVALID_ARG, "matrices of this context are still alive");
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipHostFree(ctx->pinned);
  for (int t = 0; t < bsmm_ctx_s::NSTAGE; t++) {
    if (ctx->stage_host[t]) (void)hipHostFree(ctx->stage_host[t]);
    if (ctx->stage_ev[t]) (void)hipEventDestroy(ctx->stage_ev[t]);
  }
  delete ctx;
  ABI_END
}

bsmm_status bsmm_mat_create(bsmm_ctx ctx, int32_t nbr, int32_t nbc, const int32_t *rbs, const int32_t *cbs,
                            int64_t nnzb, const int64_t *row_ptr, const int32_t *col_idx, double *values_dev,
                            int64_t n_values, bsmm_mat *out) {
  ABI_BEGIN
  if (!ctx || !out) fail(BSMM_ERR_INVALID_ARG, "ctx/out is NULL");
  if (nbr < 0 || nbc < 0 || nnzb < 0 || n_values < 0) fail(BSMM_ERR_INVALID_ARG, "negative size");
  if ((nbr > 0 && !rbs) || (nbc > 0 && !cbs) || !row_ptr || (nnzb > 0 && !col_idx))
    fail(BSMM_ERR_INVALID_ARG, "index array is NULL");
  if (n_values > 0 && !values_dev) fail(BSMM_ERR_INVALID_ARG, "values_dev is NULL");
  if (nnzb > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "more than 2^31 blocks");
  for (int32_t i = 0; i < nbr; i++) if (rbs[i] < 1) fail(BSMM_ERR_BAD_INDEX, "row block size < 1");
  for (int32_t j = 0; j < nbc; j++) if (cbs[j] < 1) fail(BSMM_ERR_BAD_INDEX, "column block size < 1");
  if (row_ptr[0] != 0) fail(BSMM_ERR_BAD_INDEX, "row_ptr[0] != 0");
  if (row_ptr[nbr] != nnzb) fail(BSMM_ERR_BAD_INDEX, "row_ptr[nbr] != nnzb");
  std::vector<int64_t> off((size_t)nnzb + 1);
  int64_t o = 0;
  for (int32_t i = 0; i < nbr; i++) {
    if (row_ptr[i + 1] < row_ptr[i]) fail(BSMM_ERR_BAD_INDEX, "row_ptr decreases");
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      int32_t j = col_idx[p];
      if (j < 0 || j >= nbc) fail(BSMM_ERR_BAD_INDEX, "col_idx out of range");
      if (p > row_ptr[i] && col_idx[p - 1] >= j) fail(BSMM_ERR_BAD_INDEX, "col_idx not strictly increasing in a row");
      off[p] = o;
      o += (int64_t)rbs[i] * cbs[j];
    }
  }
  off[nnzb] = o;
  if (o != n_values) fail(BSMM_ERR_BAD_INDEX, "n_values differs from the sum of block areas");
  DeviceGuard g(ctx->device);
  auto *m = new bsmm_mat_s();
  m->ctx = ctx;
  m->nbr = nbr;
  m->nbc = nbc;
  m->nnzb = nnzb;
  m->n_values = n_values;
  m->h_rbs.assign(rbs, rbs + nbr);
  m->h_cbs.assign(cbs, cbs + nbc);
  Allocator &al = ctx->alloc;
  try {
    m->d_rbs = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<size_t>(nbr, 1)));
    m->d_cbs = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<size_t>(nbc, 1)));
    m->d_row_ptr = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)nbr + 1)));
    m->d_col_idx = static_cast<int32_t *>(al.alloc(sizeof(int32_t) * std::max<size_t>(nnzb, 1)));
    m->d_blk_off = static_cast<int64_t *>(al.alloc(sizeof(int64_t) * ((size_t)nnzb + 1)));
    upload(m->d_rbs, rbs, sizeof(int32_t) * nbr, ctx->stream);
    upload(m->d_cbs, cbs, sizeof(int32_t) * nbc, ctx->stream);
    upload(m->d_row_ptr, row_ptr, sizeof(int64_t) * ((size_t)nbr + 1), ctx->stream);
    upload(m->d_col_idx, col_idx, sizeof(int32_t) * nnzb, ctx->stream);
    upload(m->d_blk_off, off.data(), sizeof(int64_t) * ((size_t)nnzb + 1), ctx->stream);
    // the host arrays are pageable: finish the copies before returning
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    m->owns_values = false;
    free_mat(m);
    throw;
  }
  m->d_values = values_dev;
  m->owns_values = false;
  ctx->live_mats++;
  *out = m;
  ABI_END
}

bsmm_status bsmm_mat_info(bsmm_mat m, int32_t *nbr, int32_t *nbc, int64_t *nnzb, int64_t *n_values) {
  ABI_BEGIN
  if (!m) fail(BSMM_ERR_INVALID_ARG, "m is NULL");
  if (nbr) *nbr = m->nbr;
  if (nbc) *nbc = m->nbc;
  if (nnzb) *nnzb = m->nnzb;
  if (n_values) *n_values = m->n_values;
  ABI_END
}

bsmm_status bsmm_mat_get_index(bsmm_mat m, int64_t *row_ptr, int32_t *col_idx) {
  ABI_BEGIN
  if (!m || !row_ptr || (m->nnzb > 0 && !col_idx)) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard g(m->ctx->device);
  hipStream_t s = m->ctx->stream;
  HIPCHECK(hipMemcpyAsync(row_ptr, m->d_row_ptr, sizeof(int64_t) * ((size_t)m->nbr + 1), hipMemcpyDeviceToHost, s));
  if (m->nnzb > 0)
    HIPCHECK(hipMemcpyAsync(col_idx, m->d_col_idx, sizeof(int32_t) * (size_t)m->nnzb, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  ABI_END
}

bsmm_status bsmm_mat_get_block_sizes(bsmm_mat m, int32_t *rbs, int32_t *cbs) {
  ABI_BEGIN
  if (!m || (m->nbr > 0 && !rbs) || (m->nbc > 0 && !cbs)) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (m->nbr) std::memcpy(rbs, m->h_rbs.data(), sizeof(int32_t) * m->nbr);
  if (m->nbc) std::memcpy(cbs, m->h_cbs.data(), sizeof(int32_t) * m->nbc);
  ABI_END
}

bsmm_status bsmm_mat_values(bsmm_mat m, double **values_dev) {
  ABI_BEGIN
  if (!m || !values_dev) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  *values_dev = m->d_values;
  ABI_END
}

bsmm_status bsmm_mat_copy_values(bsmm_mat m, double *dst) {
  ABI_BEGIN
  if (!m || (m->n_values > 0 && !dst)) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard g(m->ctx->device);
  if (m->n_values > 0)
    HIPCHECK(hipMemcpyAsync(dst, m->d_values, sizeof(double) * (size_t)m->n_values, hipMemcpyDeviceToDevice,
                            m->ctx->stream));
  ABI_END
}

bsmm_status bsmm_mat_destroy(bsmm_mat m) {
  ABI_BEGIN
  if (!m) fail(BSMM_ERR_INVALID_ARG, "m is NULL");
  DeviceGuard g(m->ctx->device);
  bsmm_ctx ctx = m->ctx;
  bool user = !m->owns_values;
  free_mat(m);
  (void)user;
  ctx->live_mats--;
  ABI_END
}

bsmm_status bsmm_block_norms(bsmm_mat m, double *norms) {
  ABI_BEGIN
  if (!m || (m->nnzb > 0 && !norms)) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard g(m->ctx->device);
  block_norms(*m, norms, m->ctx->stream);
  ABI_END
}

bsmm_status bsmm_multiply(bsmm_ctx ctx, char transa, char transb, double alpha, bsmm_mat a, bsmm_mat b,
                          double beta, bsmm_mat c_old, double filter_eps, int retain_sparsity, bsmm_mat *c_out,
                          bsmm_multiply_info *info) {
  ABI_BEGIN
  if (!ctx || !a || !b || !c_out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (!(transa == 'N' || transa == 'n' || transa == 'T' || transa == 't') ||
      !(transb == 'N' || transb == 'n' || transb == 'T' || transb == 't'))
    fail(BSMM_ERR_INVALID_ARG, "trans must be 'N' or 'T'");
  if (a->ctx != ctx || b->ctx != ctx || (c_old && c_old->ctx != ctx))
    fail(BSMM_ERR_INVALID_ARG, "matrices belong to another context");
  DeviceGuard g(ctx->device);
  bsmm_mat_s *r = multiply_impl(ctx, transa, transb, alpha, a, b, beta, c_old, filter_eps, retain_sparsity, info);
  ctx->live_mats++;
  *c_out = r;
  ABI_END
}

// ------------------------------------------------------------------ plans
struct bsmm_plan_s {
  Plan plan;
  explicit bsmm_plan_s(bsmm_ctx c) : plan(c) {}
};

bsmm_status bsmm_plan_create(bsmm_ctx ctx, char transa, char transb, double alpha, bsmm_mat a, bsmm_mat b,
                             double beta, bsmm_mat c_old, double filter_eps, int retain_sparsity, bsmm_plan *out,
                             bsmm_multiply_info *info) {
  ABI_BEGIN
  if (!ctx || !a || !b || !out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (!(transa == 'N' || transa == 'n' || transa == 'T' || transa == 't') ||
      !(transb == 'N' || transb == 'n' || transb == 'T' || transb == 't'))
    fail(BSMM_ERR_INVALID_ARG, "trans must be 'N' or 'T'");
  if (a->ctx != ctx || b->ctx != ctx || (c_old && c_old->ctx != ctx))
    fail(BSMM_ERR_INVALID_ARG, "matrices belong to another context");
  DeviceGuard g(ctx->device);
  auto *pl = new bsmm_plan_s(ctx);
  try {
    Plan &P = pl->plan;
    P.A = a;
    P.B = b;
    P.C0 = c_old;
    P.alpha = alpha;
    P.beta = beta;
    P.eps = filter_eps;
    P.retain = retain_sparsity;
    plan_build(P, transa, transb);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    if (info) {
      *info = bsmm_multiply_info{};
      info->c_nnzb_symbolic = P.nnzb_c;
      info->c_nnzb = P.nnzb_c;
      info->c_n_values = P.nval_c;
      info->n_products = P.nprod;
      info->n_candidates = P.ncand;
      info->useful_flops = 2.0 * (double)P.kmn_total;
      info->ms_index = P.tm.between(0, 1);
      info->ms_norms = P.tm.between(1, 2);
      info->ms_symbolic = P.tm.between(2, 3);
      info->ms_stacks = P.tm.between(3, 4);
      info->gemm_path = gemm_path(P);
    }
  } catch (...) {
    // leave the stream idle: nothing the failed plan queued is still running
    (void)hipStreamSynchronize(ctx->stream);
    delete pl;
    throw;
  }
  ctx->live_mats++;
  *out = pl;
  ABI_END
}

bsmm_status bsmm_plan_sizes(bsmm_plan plan, int64_t *c_nnzb, int64_t *c_n_values, size_t *workspace_bytes) {
  ABI_BEGIN
  if (!plan) fail(BSMM_ERR_INVALID_ARG, "plan is NULL");
  const Plan &P = plan->plan;
  if (c_nnzb) *c_nnzb = P.nnzb_c;
  if (c_n_values) *c_n_values = P.nval_c;
  if (workspace_bytes) *workspace_bytes = P.ws.total;
  ABI_END
}

bsmm_status bsmm_plan_filter_holds(bsmm_plan plan, int32_t *holds) {
  ABI_BEGIN
  if (!plan || !holds) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  Plan &P = plan->plan;
  *holds = filter_decisions_hold(P, P.A, P.B) ? 1 : 0;
  ABI_END
}

bsmm_status bsmm_plan_execute_into(bsmm_plan plan, double *c_values_dev, void *workspace_dev, bsmm_mat *c_out) {
  ABI_BEGIN
  if (!plan || !c_out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  Plan &P = plan->plan;
  if (P.nval_c > 0 && !c_values_dev) fail(BSMM_ERR_INVALID_ARG, "c_values_dev is NULL");
  if (P.ws.total > 0 && !workspace_dev) fail(BSMM_ERR_INVALID_ARG, "workspace_dev is NULL");
  if (((uintptr_t)workspace_dev & 255u) != 0) fail(BSMM_ERR_INVALID_ARG, "workspace_dev is not 256-byte aligned");
  if (((uintptr_t)c_values_dev & 7u) != 0) fail(BSMM_ERR_INVALID_ARG, "c_values_dev is not 8-byte aligned");
  auto overlaps = [](const void *x, size_t nx, const void *y, size_t ny) {
    const char *a = static_cast<const char *>(x), *b = static_cast<const char *>(y);
    return x && y && nx && ny && a < b + ny && b < a + nx;
  };
  const size_t cb = 8 * (size_t)P.nval_c;
  for (const bsmm_mat_s *m : {P.A, P.B, P.C0}) {
    if (!m) continue;
    if (overlaps(c_values_dev, cb, m->d_values, 8 * (size_t)m->n_values) ||
        overlaps(workspace_dev, P.ws.total, m->d_values, 8 * (size_t)m->n_values))
      fail(BSMM_ERR_ALIAS, "a caller buffer overlaps the values of an operand");
  }
  if (overlaps(c_values_dev, cb, workspace_dev, P.ws.total))
    fail(BSMM_ERR_ALIAS, "c_values_dev overlaps workspace_dev");
  DeviceGuard g(P.ctx->device);
  bind_numeric(P, c_values_dev, static_cast<uint8_t *>(workspace_dev));
  P.caller_bound = true;
  plan_numeric(P, false);
  bsmm_mat_s *R = plan_finish_into(P);
  P.ctx->live_mats++;
  *c_out = R;
  ABI_END
}

bsmm_status bsmm_plan_execute(bsmm_plan plan) {
  ABI_BEGIN
  if (!plan) fail(BSMM_ERR_INVALID_ARG, "plan is NULL");
  Plan &P = plan->plan;
  DeviceGuard g(P.ctx->device);
  ensure_own_buffers(P);   // allocates before any launch of this call
  if (P.exec)
    HIPCHECK(hipGraphLaunch(P.exec, P.ctx->stream));
  else
    plan_numeric(P, false);
  ABI_END
}

bsmm_status bsmm_plan_capture(bsmm_plan plan) {
  ABI_BEGIN
  if (!plan) fail(BSMM_ERR_INVALID_ARG, "plan is NULL");
  Plan &P = plan->plan;
  if (P.exec) return BSMM_OK;   // already captured
  if (P.ctx->stream == nullptr) fail(BSMM_ERR_UNSUPPORTED, "graph capture needs a non-default stream");
  DeviceGuard g(P.ctx->device);
  ensure_own_buffers(P);   // no allocation under capture
  HIPCHECK(hipStreamBeginCapture(P.ctx->stream, hipStreamCaptureModeThreadLocal));
  try {
    plan_numeric(P, false);
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(P.ctx->stream, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(P.ctx->stream, &P.graph));
  HIPCHECK(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  ABI_END
}

bsmm_status bsmm_plans_execute(int32_t n, bsmm_plan *plans) {
  ABI_BEGIN
  if (n < 0 || (n > 0 && !plans)) fail(BSMM_ERR_INVALID_ARG, "bad plan list");
  if (n == 0) return BSMM_OK;
  bsmm_ctx ctx = nullptr;
  for (int32_t r = 0; r < n; r++) {
    if (!plans[r]) fail(BSMM_ERR_INVALID_ARG, "plan is NULL");
    if (r == 0) ctx = plans[0]->plan.ctx;
    if (plans[r]->plan.ctx != ctx) fail(BSMM_ERR_INVALID_ARG, "plans of different contexts");
    for (int32_t q = 0; q < r; q++)
      if (plans[q] == plans[r]) fail(BSMM_ERR_INVALID_ARG, "a plan appears twice");
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  bool batched = true;
  for (int32_t r = 0; r < n; r++) batched = batched && plans[r]->plan.quads && !plans[r]->plan.lowp;
  if (!batched) {   // one after another, as bsmm_plan_execute
    for (int32_t r = 0; r < n; r++) ensure_own_buffers(plans[r]->plan);
    for (int32_t r = 0; r < n; r++) {
      Plan &P = plans[r]->plan;
      if (P.exec) HIPCHECK(hipGraphLaunch(P.exec, s));
      else plan_numeric(P, false);
    }
    return BSMM_OK;
  }
  std::vector<const GemmArgs *> gs;
  std::vector<int64_t> nnzb;
  int max_edge = 1;
  for (int32_t r = 0; r < n; r++) ensure_own_buffers(plans[r]->plan);   // every allocation before any launch
  for (int32_t r = 0; r < n; r++) {
    Plan &P = plans[r]->plan;
    if (P.nprod > 0)
      pack_values(*P.A, P.ta, P.a_poff.p, const_cast<double *>(P.ga.a_pack), *P.B, !P.tb, P.b_poff.p,
                  const_cast<double *>(P.ga.b_pack), s);
    gs.push_back(&P.ga);
    nnzb.push_back(P.nnzb_c);
    max_edge = std::max(max_edge, P.max_edge);
  }
  // launch parameters go through a ring of pinned host slots: a slot is
  // rewritten once the copy out of it has run (its event), so the host never
  // waits for the GEMM itself; the device buffer is reused in stream order
  const size_t need = gemm_multi_stage_bytes(n);
  if (need > ctx->batch_bytes) {
    (void)hipStreamSynchronize(s);   // no copy from the old slots is pending
    for (int t = 0; t < bsmm_ctx_s::NSTAGE; t++) {
      if (ctx->stage_host[t]) (void)hipHostFree(ctx->stage_host[t]);
      ctx->stage_host[t] = nullptr;
    }
    ctx->alloc.release(ctx->batch_dev);
    ctx->batch_dev = nullptr;
    ctx->batch_bytes = 0;
    const size_t cap = std::max<size_t>(need, 64 * 1024);
    for (int t = 0; t < bsmm_ctx_s::NSTAGE; t++) {
      if (hipHostMalloc(&ctx->stage_host[t], cap, hipHostMallocDefault) != hipSuccess) {
        ctx->stage_host[t] = nullptr;
        fail(BSMM_ERR_OUT_OF_MEMORY, "pinned staging buffer");
      }
      if (!ctx->stage_ev[t]) HIPCHECK(hipEventCreateWithFlags(&ctx->stage_ev[t], hipEventDisableTiming));
    }
    ctx->batch_dev = ctx->alloc.alloc(cap);
    ctx->batch_bytes = cap;
  }
  const int slot = ctx->stage_next;
  HIPCHECK(hipEventSynchronize(ctx->stage_ev[slot]));   // the copy out of this slot has run
  gemm_launch_multi(ctx->alloc, gs, nnzb, max_edge, ctx->stage_host[slot], ctx->batch_bytes, ctx->batch_dev, s);
  HIPCHECK(hipEventRecord(ctx->stage_ev[slot], s));
  ctx->stage_next = (slot + 1) % bsmm_ctx_s::NSTAGE;
  ABI_END
}

bsmm_status bsmm_plan_result(bsmm_plan plan, bsmm_mat *c_out) {
  ABI_BEGIN
  if (!plan || !c_out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  Plan &P = plan->plan;
  DeviceGuard g(P.ctx->device);
  bsmm_mat_s *r = plan_finish(P, false);
  P.ctx->live_mats++;
  *c_out = r;
  ABI_END
}

bsmm_status bsmm_plan_destroy(bsmm_plan plan) {
  ABI_BEGIN
  if (!plan) return BSMM_OK;
  bsmm_ctx ctx = plan->plan.ctx;
  DeviceGuard g(ctx->device);
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  delete plan;
  ctx->live_mats--;
  ABI_END
}

bsmm_status bsmm_sign_newton_schulz(bsmm_ctx ctx, bsmm_mat x0, int32_t max_iter, double filter_eps, double tol,
                                    bsmm_mat *x_out, bsmm_sign_info *info, double *trace_residual,
                                    int64_t *trace_nnzb) {
  ABI_BEGIN
  if (!ctx || !x0 || !x_out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (x0->ctx != ctx) fail(BSMM_ERR_INVALID_ARG, "matrix belongs to another context");
  DeviceGuard g(ctx->device);
  bsmm_mat_s *r = sign_impl(ctx, x0, max_iter, filter_eps, tol, info, trace_residual, trace_nnzb);
  ctx->live_mats++;
  *x_out = r;
  ABI_END
}

bsmm_status bsmm_filter(bsmm_mat m, double eps, bsmm_mat *out) {
  ABI_BEGIN
  if (!m || !out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (!(eps >= 0.0)) fail(BSMM_ERR_INVALID_ARG, "eps must be >= 0");
  bsmm_ctx ctx = m->ctx;
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  Allocator &al = ctx->alloc;
  const size_t n1 = (size_t)std::max<int64_t>(m->nnzb, 1);
  DBuf<double> norm(al, n1);
  DBuf<int32_t> flags(al, n1);
  block_norms(*m, norm.p, s);
  CompactArgs ca;
  ca.nbr = m->nbr;
  ca.nnzb = m->nnzb;
  ca.rp = m->d_row_ptr;
  ca.ci = m->d_col_idx;
  ca.off = m->d_blk_off;
  ca.values = m->d_values;
  ca.norm = norm.p;
  ca.eps = eps;
  DBuf<int64_t> rank;
  int64_t kept = count_kept(al, ca, flags.p, ctx->pinned, s, rank);
  bsmm_mat_s *R = new_result(ctx, m->nbr, m->nbc, m->h_rbs, m->h_cbs);
  try {
    DBuf<int64_t> nrp(al, (size_t)m->nbr + 1), noff(al, (size_t)std::max<int64_t>(kept, 1) + 1);
    DBuf<int32_t> nci(al, (size_t)std::max<int64_t>(kept, 1));
    double *nv = nullptr;
    int64_t nval = 0;
    compact(al, ca, rank.p, m->d_rbs, m->d_cbs, nrp.p, nci.p, noff.p, ctx->pinned, &nv, &nval, s);
    R->d_row_ptr = nrp.release_ownership();
    R->d_col_idx = nci.release_ownership();
    R->d_blk_off = noff.release_ownership();
    R->d_values = nv;
    R->nnzb = kept;
    R->n_values = nval;
  } catch (...) {
    free_mat(R);
    throw;
  }
  ctx->live_mats++;
  *out = R;
  ABI_END
}

}  // extern "C"
