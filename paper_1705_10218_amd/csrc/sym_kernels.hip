// sym_kernels.hip -- symbolic phase (block pattern of C), product counts per
// C block, and stack generation.
//
// The result pattern is not known in advance (arXiv:1705.10218, Section 2):
// block (i,j) of C exists when some k has A(i,k) and B(k,j) stored (plus
// C_old's blocks when beta != 0, or exactly C_old's under retain_sparsity).
// One workgroup owns one block row i of C and marks the reachable block
// columns in a bitmap held in LDS; the bitmap doubles as the map from a
// block column to its position inside the row (prefix popcounts), so
// neither a dense column map nor a sort is needed.
#include <type_traits>

#include "internal.h"

namespace bsmm {

namespace {

constexpr int SYM_THREADS = 256;
constexpr int32_t MAX_WORDS = 4096;      // bitmap window: 131072 block columns
constexpr int32_t CNT_CAP = 8192;        // per-row counters kept in LDS up to this
constexpr int MAX_KSIZES = 8;            // k-size grouping of the stacks up to this many sizes
constexpr size_t STACK_LDS_HEAD = 1792;  // stack fill: 64 opened A entries (B row start, norm, count, A half, k bits)
constexpr int64_t STACK_BUF_BYTES = 16384;  // windowed stack fill: LDS for buffered entries (32 B per C block)

// Distinct k block sizes, ascending (nks == 0: no grouping by size).
struct KSizes {
  int32_t v[MAX_KSIZES];
};

struct OpView {
  const int64_t *rp;
  const int32_t *ci;
  const int32_t *blk;   // null = identity
  const int32_t *rbs, *cbs;
  const int64_t *off;   // value offsets of the original blocks
};

OpView view(const OpIndex &o) { return OpView{o.row_ptr, o.col_idx, o.blk, o.rbs, o.cbs, o.blk_off}; }

__device__ inline void bm_set(uint32_t *bm, int32_t j) { atomicOr(&bm[j >> 5], 1u << (j & 31)); }
__device__ inline bool bm_test(const uint32_t *bm, int32_t j) { return (bm[j >> 5] >> (j & 31)) & 1u; }
__device__ inline int32_t bm_slot(const uint32_t *bm, const int32_t *pre, int32_t j) {
  uint32_t w = bm[j >> 5];
  return pre[j >> 5] + __popc(w & ((1u << (j & 31)) - 1u));
}

// position of j in the sorted slice ci[lo, hi), or -1
__device__ inline int32_t bsearch_slot(const int32_t *ci, int64_t lo, int64_t hi, int32_t j) {
  int64_t base = lo;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    int32_t v = ci[mid];
    if (v == j) return (int32_t)(mid - base);
    if (v < j) lo = mid + 1; else hi = mid;
  }
  return -1;
}

template <typename T>
__device__ inline T block_sum(T v, T *sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T t = 0;
  for (int q = 0; q < nw; q++) t += sh[q];
  __syncthreads();
  return t;
}

// Mark every candidate block column of row i that falls in [j0, j1).
// One record per entry q of op(B): the block column, the B half of a stack
// entry (byte offset into the packed copy, or the block id) and the block
// norm, so a product costs one 16-byte load on the B side.
struct alignas(16) BEnt {
  int32_t j;
  uint32_t eb;
  double nb;
};

// Up to 64 opened A entries of one block row, staged in LDS per wavefront.
struct AOpen {
  int64_t qb[64];   // first entry of B row k
  double na[64];    // norm of A(i,k) (0 without filter)
  int32_t nq[64];   // entries of B row k (> 0)
  int32_t kk[64];   // k block size
  int32_t kx[64];   // index of the k size in the size list (0 without grouping)
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Opens A entries p0 + lane (below p1), one per lane: those with a non-empty
// B row are compacted into st in ascending order.  Returns their number;
// adds each lane's candidate products (entries of its B row) to *cand.
__device__ inline int open_a(const OpView &A, const OpView &B, int64_t p0, int64_t p1, const double *na,
                             const KSizes *ksz, int nkp, AOpen &st, int64_t *cand) {
  const int lane = threadIdx.x & 63;
  const int64_t p = p0 + lane;
  bool ok = false;
  int64_t qb = 0;
  int32_t nq = 0, kk = 0, kx = 0;
  double nA = 0.0;
  if (p < p1) {
    const int32_t k = A.ci[p];
    kk = A.cbs[k];
    qb = B.rp[k];
    nq = (int32_t)(B.rp[k + 1] - qb);
    ok = nq > 0;
    if (na) nA = na[A.blk ? A.blk[p] : (int32_t)p];
    if (nkp > 0)
      while (kx + 1 < nkp && ksz->v[kx] != kk) kx++;
  }
  if (cand) *cand += nq;
  const uint64_t m = __ballot(ok);
  if (ok) {
    const int t = __popcll(m & ((1ull << lane) - 1ull));
    st.qb[t] = qb;
    st.na[t] = nA;
    st.nq[t] = nq;
    st.kk[t] = kk;
    st.kx[t] = kx;
  }
  return __popcll(m);
}

// Visits the products of the opened entries of one wavefront (B row starts
// qb[e], lengths nq[e], e < ne) in chunks of up to 64 consecutive entries
// of one B row, a lane per product, in ascending (entry, q) order, calling
// f(e, load(q)) on the lanes that hold a product.  D chunks are
// loaded back to back (every lane loads; a lane without a product loads
// item 0, so no branch separates the loads) before they are handled: one
// memory latency per D chunks.  load(0) must be a valid item
// whenever some opened entry exists.
constexpr int WALK_DEPTH = 8;

template <typename T, int D = WALK_DEPTH, typename L, typename F>
__device__ inline void chunk_walk(const int64_t *qb, const int32_t *nq, int ne, L load, F f) {
  const int lane = threadIdx.x & 63;
  int e = 0;   // next chunk: entry e, offset o
  int32_t o = 0;
  while (e < ne) {
    int pe[D];
    bool pv[D];
    T v[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
      const bool live = e < ne;   // uniform
      const int es = live ? e : 0;
      const int32_t n = nq[es];
      pe[d] = es;
      pv[d] = live && o + lane < n;
      v[d] = load(pv[d] ? qb[es] + o + lane : (int64_t)0);
      if (live) {
        o += 64;
        if (o >= n) {
          e++;
          o = 0;
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; d++)
      if (pv[d]) f(pe[d], v[d]);
  }
}

// Marks the block columns in [j0, j1) reachable from row i of A.  Each
// wavefront opens every (nw*64)-th batch of the row's A entries.
__device__ inline void mark_candidates(const OpView &A, const OpView &B, int32_t i, int32_t j0, int32_t j1,
                                       uint32_t *bm, AOpen *stage) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  AOpen &st = stage[wv];
  const int64_t pa1 = A.rp[i + 1];
  for (int64_t pb = A.rp[i] + (int64_t)wv * 64; pb < pa1; pb += (int64_t)nw * 64) {
    const int ne = open_a(A, B, pb, pa1, nullptr, nullptr, 0, st, nullptr);
    wave_sync();
    chunk_walk<int32_t>(st.qb, st.nq, ne, [&](int64_t q) { return B.ci[q]; }, [&](int, int32_t j) {
      if (j >= j0 && j < j1) bm_set(bm, j - j0);
    });
    wave_sync();
  }
}

__device__ inline void mark_row(const int64_t *rp, const int32_t *ci, int32_t i, int32_t j0, int32_t j1,
                                uint32_t *bm) {
  for (int64_t q = rp[i] + threadIdx.x; q < rp[i + 1]; q += blockDim.x) {
    int32_t j = ci[q];
    if (j >= j0 && j < j1) bm_set(bm, j - j0);
  }
}

// Work unit of a workgroup in the row-parallel kernels.  A launch has
// 8 * per_xcd workgroups, which the hardware deals to the 8 XCDs
// round-robin; unit ids are remapped so that each XCD takes one contiguous
// stretch of rows, in the locality order ord when given (nu units per row),
// and its L2 holds the op(B) rows that stretch needs.  ok = false for the
// padding workgroups past the last unit.
struct RowUnit {
  int32_t row;
  int unit;
  bool ok;
};

__device__ inline RowUnit row_unit(int32_t nrows, int nu, int64_t per_xcd, const int32_t *ord) {
  const int64_t b = blockIdx.x;
  const int64_t id = (b & 7) * per_xcd + (b >> 3);
  RowUnit r{0, 0, id < (int64_t)nrows * nu};
  if (r.ok) {
    const int32_t pos = (int32_t)(id / nu);
    r.unit = (int)(id - (int64_t)pos * nu);
    r.row = ord ? ord[pos] : pos;
  }
  return r;
}

inline int64_t row_units_per_xcd(int32_t nrows, int nu) { return ((int64_t)nrows * nu + 7) / 8; }

// Exclusive prefix popcount over W words (block-wide, simple two-level).
__device__ inline void word_prefix(const uint32_t *bm, int32_t *pre, int32_t W, int32_t *sh) {
  int t = threadIdx.x, nt = blockDim.x;
  int32_t per = (W + nt - 1) / nt;
  int32_t w0 = t * per, w1 = min(W, w0 + per);
  int32_t s = 0;
  for (int32_t w = w0; w < w1; w++) s += __popc(bm[w]);
  // exclusive scan of s over threads
  int lane = t & 63, wv = t >> 6, nw = nt >> 6;
  int32_t inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  __syncthreads();
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  int32_t base = 0;
  for (int q = 0; q < wv; q++) base += sh[q];
  int32_t run = base + inc - s;
  for (int32_t w = w0; w < w1; w++) {
    pre[w] = run;
    run += __popc(bm[w]);
  }
  (void)nw;
  __syncthreads();
}

// ------------------------------------------------------------ a2: count
__global__ __launch_bounds__(SYM_THREADS) void k_sym_count(OpView A, OpView B, const int64_t *cold_rp,
                                                           const int32_t *cold_ci, int use_cold, int32_t nbc,
                                                           int64_t *row_nnz, int32_t *max_row, int32_t nbr,
                                                           const int32_t *ord, int64_t per_xcd, uint32_t *gbits) {
  extern __shared__ uint32_t bm[];
  __shared__ int64_t red[SYM_THREADS / 64];
  __shared__ AOpen stage[SYM_THREADS / 64];
  const RowUnit ru = row_unit(nbr, 1, per_xcd, ord);
  if (!ru.ok) return;
  const int32_t i = ru.row;
  int32_t words_total = (nbc + 31) >> 5;
  if (words_total == 0) {
    if (threadIdx.x == 0) row_nnz[i] = 0;
    return;
  }
  int32_t W = min(words_total, MAX_WORDS);
  int32_t nwin = (words_total + W - 1) / W;
  int64_t total = 0;
  for (int32_t win = 0; win < nwin; win++) {
    int32_t j0 = win * W * 32, j1 = min(nbc, j0 + W * 32);
    for (int32_t t = threadIdx.x; t < W; t += blockDim.x) bm[t] = 0u;
    __syncthreads();
    if (use_cold) mark_row(cold_rp, cold_ci, i, j0, j1, bm);
    mark_candidates(A, B, i, j0, j1, bm, stage);
    __syncthreads();
    int64_t c = 0;
    for (int32_t t = threadIdx.x; t < W; t += blockDim.x) {
      c += __popc(bm[t]);
      if (gbits) gbits[(int64_t)i * W + t] = bm[t];   // kept for the fill (single window)
    }
    total += block_sum<int64_t>(c, red);
  }
  if (threadIdx.x == 0) {
    row_nnz[i] = total;
    if (max_row) atomicMax(max_row, (int32_t)total);
  }
}

// ------------------------------------------- a2 fill + a4 product counts
// Writes C's col_idx for row i, the block row / size of every C block, the
// number of products per C block that pass the on-the-fly filter
// (kept iff !(||A_ik|| * ||B_kj|| < eps)) and the row's sum of k over kept
// products (for the useful flop count).
__global__ __launch_bounds__(SYM_THREADS) void k_sym_fill(OpView A, OpView B, const int64_t *cold_rp,
                                                          const int32_t *cold_ci, int use_cold, int retain,
                                                          int32_t nbc, const int64_t *c_rp, int32_t *c_ci,
                                                          int32_t *c_row, int64_t *c_size, int32_t *c_cnt,
                                                          int64_t *row_kmn, int64_t *row_cand, int64_t *row_real,
                                                          const BEnt *bent, const double *na, double eps,
                                                          int32_t cnt_cap, KSizes ksz, int nkp, int32_t *cnt_g,
                                                          int32_t *kofs, int32_t nbr, const int32_t *ord,
                                                          int64_t per_xcd, const uint32_t *gbits, int diag8,
                                                          unsigned long long *margin) {
  extern __shared__ uint32_t sm[];
  __shared__ int32_t shi[SYM_THREADS / 64];
  __shared__ int64_t shl[SYM_THREADS / 64];
  __shared__ AOpen stage[SYM_THREADS / 64];
  const RowUnit ru = row_unit(nbr, 1, per_xcd, ord);
  if (!ru.ok) return;
  const int32_t i = ru.row;
  int32_t words_total = (nbc + 31) >> 5;
  if (words_total == 0) {
    if (threadIdx.x == 0) { row_kmn[i] = 0; row_cand[i] = 0; row_real[i] = 0; }
    return;
  }
  int32_t W = min(words_total, MAX_WORDS);
  int32_t nwin = (words_total + W - 1) / W;
  uint32_t *bm = sm;
  int32_t *pre = reinterpret_cast<int32_t *>(sm + W);
  int32_t *cnt = pre + W;
  const int64_t cbase = c_rp[i];
  const int32_t R = (int32_t)(c_rp[i + 1] - cbase);
  const int32_t m = A.rbs[i];
  int64_t wbase = cbase;
  for (int32_t win = 0; win < nwin; win++) {
    int32_t j0 = win * W * 32, j1 = min(nbc, j0 + W * 32);
    if (gbits) {   // the counting pass's bitmap of this row (single window)
      for (int32_t t = threadIdx.x; t < W; t += blockDim.x) bm[t] = gbits[(int64_t)i * W + t];
    } else {
      for (int32_t t = threadIdx.x; t < W; t += blockDim.x) bm[t] = 0u;
      __syncthreads();
      if (retain) {
        mark_row(cold_rp, cold_ci, i, j0, j1, bm);
      } else {
        if (use_cold) mark_row(cold_rp, cold_ci, i, j0, j1, bm);
        mark_candidates(A, B, i, j0, j1, bm, stage);
      }
    }
    __syncthreads();
    word_prefix(bm, pre, W, shi);
    for (int32_t t = threadIdx.x; t < W; t += blockDim.x) {
      uint32_t w = bm[t];
      int64_t pos = wbase + pre[t];
      while (w) {
        int b = __ffs(w) - 1;
        w &= w - 1u;
        int32_t j = j0 + t * 32 + b;
        c_ci[pos] = j;
        c_row[pos] = i;
        c_size[pos] = (int64_t)m * B.cbs[j];
        pos++;
      }
    }
    int32_t last = W - 1;
    int64_t wcount = (int64_t)pre[last] + __popc(bm[last]);
    __syncthreads();
    wbase += wcount;
  }
  // counts of kept products per C block, per k size when padding (nkp > 0):
  // every run of equal k size is padded to a multiple of 4 entries
  const bool lds_slot = (nwin == 1);
  const int nk1 = nkp > 0 ? nkp : 1;
  const bool lds_cnt = ((int64_t)R * nk1 <= cnt_cap);
  int32_t *gcnt = nkp > 0 ? cnt_g + cbase * nk1 : c_cnt + cbase;
  if (lds_cnt)
    for (int32_t t = threadIdx.x; t < R * nk1; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t kmn = 0, cand = 0;
  // filter margins: the smallest kept and the largest dropped norm product
  double kept_min = INFINITY, drop_max = 0.0;
  {
    AOpen &st = stage[wv];
    const int64_t pa1 = A.rp[i + 1];
    for (int64_t pb = A.rp[i] + (int64_t)wv * 64; pb < pa1; pb += (int64_t)nw * 64) {
      const int ne = open_a(A, B, pb, pa1, na, &ksz, nkp, st, &cand);
      wave_sync();
      auto walk = [&](auto fast) {
        constexpr bool FAST = decltype(fast)::value;
        chunk_walk<BEnt>(st.qb, st.nq, ne, [&](int64_t q) { return bent[q]; }, [&](int e, const BEnt &v) {
          if (na) {
            const double pr = st.na[e] * v.nb;
            if (pr < eps) {
              drop_max = fmax(drop_max, pr);
              return;
            }
            kept_min = fmin(kept_min, pr);
          }
          if constexpr (FAST) {
            if (!bm_test(bm, v.j)) return;   // only under retain_sparsity
            atomicAdd(&cnt[bm_slot(bm, pre, v.j) * nk1 + st.kx[e]], 1);
          } else {
            int32_t slot;
            if (lds_slot) slot = bm_test(bm, v.j) ? bm_slot(bm, pre, v.j) : -1;
            else slot = bsearch_slot(c_ci, cbase, cbase + R, v.j);
            if (slot < 0) return;
            const int kx = st.kx[e];
            if (lds_cnt) atomicAdd(&cnt[slot * nk1 + kx], 1);
            else atomicAdd(&gcnt[slot * nk1 + kx], 1);
            if (nkp == 0) kmn += (int64_t)st.kk[e] * B.cbs[v.j];
          }
        });
      };
      // slots and counters in LDS with k sizes known per run: a loop with no
      // global load besides the ring's
      if (lds_slot && lds_cnt && nkp > 0) walk(std::true_type{});
      else walk(std::false_type{});
      wave_sync();
    }
  }
  __syncthreads();
  // per C block: run starts of its k sizes, padded and kept counts; with k
  // sizes known per run, its share of the useful flops (sum of k * n)
  int64_t real = 0;
  for (int32_t t = threadIdx.x; t < R; t += blockDim.x) {
    int32_t tot_real = 0, tot_pad = 0;
    int64_t ksum = 0;
    // runs padded to groups of four products, of eight for the blocks of the
    // diagonal-packed GEMM variant (both edges at most 8)
    const int32_t gm = (diag8 && m <= 8 && B.cbs[c_ci[cbase + t]] <= 8) ? 7 : 3;
    for (int kx = 0; kx < nk1; kx++) {
      const int32_t v = lds_cnt ? cnt[t * nk1 + kx] : gcnt[t * nk1 + kx];
      if (kofs) kofs[(cbase + t) * nk1 + kx] = tot_pad;   // this k size's run starts here
      tot_real += v;
      tot_pad += nkp > 0 ? (v + gm) & ~gm : v;
      if (nkp > 0) ksum += (int64_t)v * ksz.v[kx];
    }
    c_cnt[cbase + t] = tot_pad;
    real += tot_real;
    if (nkp > 0) kmn += ksum * B.cbs[c_ci[cbase + t]];
  }
  if (margin && na) {   // non-negative doubles order like their bit patterns
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      kept_min = fmin(kept_min, __shfl_xor(kept_min, d, 64));
      drop_max = fmax(drop_max, __shfl_xor(drop_max, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&margin[0], (unsigned long long)__double_as_longlong(kept_min));
      atomicMax(&margin[1], (unsigned long long)__double_as_longlong(drop_max));
    }
  }
  int64_t tot = block_sum<int64_t>(kmn, shl);
  int64_t tcand = block_sum<int64_t>(cand, shl);
  int64_t treal = block_sum<int64_t>(real, shl);
  if (threadIdx.x == 0) {
    row_kmn[i] = tot * m;
    row_cand[i] = tcand;
    row_real[i] = treal;
  }
}

// ----------------------------------------------------- C_old block map
__global__ void k_old_map(const int64_t *cold_rp, const int32_t *cold_ci, const int64_t *c_rp,
                          const int32_t *c_ci, int32_t *old_blk) {
  int32_t i = blockIdx.x;
  int64_t c0 = c_rp[i], c1 = c_rp[i + 1];
  for (int64_t q = cold_rp[i] + threadIdx.x; q < cold_rp[i + 1]; q += blockDim.x) {
    int32_t s = bsearch_slot(c_ci, c0, c1, cold_ci[q]);
    if (s >= 0) old_blk[c0 + s] = (int32_t)q;
  }
}

// ------------------------------------------------------ a4: stack fill
__global__ __launch_bounds__(256) void k_product_records(OpView B, int64_t nq, const double *nb, int enc,
                                                         const int64_t *b_base, BEnt *out) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t bblk = B.blk ? B.blk[q] : (int32_t)q;
    BEnt e;
    e.j = B.ci[q];
    e.eb = enc ? (uint32_t)((B.off[bblk] - (b_base ? b_base[e.j] : 0)) * 8) : (uint32_t)bblk;
    e.nb = nb ? nb[bblk] : 0.0;
    out[q] = e;
  }
}

// One wavefront per (C block row i, k size): the k-size runs of a segment
// are independent (their starts come from the symbolic phase), so the
// passes of a row run side by side.  The A entries of row i are opened 64 at
// a time, one per lane (k, the range of B row k, the norm and the A half of
// the entry); those of this pass's k size with a non-empty B row are
// compacted into LDS in ascending k.  Their products are then taken in
// chunks of up to 64 consecutive entries of one B row, a lane per product.
// A given block column appears once in a B row, so the per-C-block write
// cursors (in LDS, beside the run starts) never collide inside a chunk, and
// chunks go in ascending k: every C block's run comes out sorted by k,
// identically on every run.
__global__ __launch_bounds__(64) void k_stack_fill(OpView A, OpView B, int32_t nbc, const int64_t *c_rp,
                                                   const int32_t *c_ci, const int64_t *seg_off,
                                                   const int32_t *kofs, int2 *stack, const BEnt *bent,
                                                   const double *na, double eps, int32_t cnt_cap, int32_t *run,
                                                   KSizes ksz, int nks, int pad4, int enc, int32_t nbr,
                                                   const int32_t *ord, int64_t per_xcd, int diag8,
                                                   const int64_t *a_base) {
  extern __shared__ uint32_t sm[];
  const RowUnit ru = row_unit(nbr, nks > 0 ? nks : 1, per_xcd, ord);
  if (!ru.ok) return;
  const int32_t i = ru.row;
  const int pass = ru.unit;   // k-size index (0 when nks == 0)
  const int lane = threadIdx.x;
  const int32_t words_total = (nbc + 31) >> 5;
  const int32_t W = min(words_total, MAX_WORDS);
  const bool lds_slot = words_total <= MAX_WORDS;
  const int64_t cbase = c_rp[i];
  const int32_t R = (int32_t)(c_rp[i + 1] - cbase);
  if (R == 0) return;
  const bool lds_cnt = R <= cnt_cap;
  const int nk1 = nks > 0 ? nks : 1;
  const int64_t abase = a_base ? a_base[i] : 0;   // encoded A offsets start at row i's packed blocks
  // opened A entries (64 at most at a time)
  int64_t *s_qb = reinterpret_cast<int64_t *>(sm);
  double *s_na = reinterpret_cast<double *>(sm + 128);
  int32_t *s_nq = reinterpret_cast<int32_t *>(sm + 256);
  uint32_t *s_ea = sm + 320;
  uint32_t *s_kb = sm + 384;
  uint32_t *bm = sm + STACK_LDS_HEAD / 4;
  int32_t *pre = reinterpret_cast<int32_t *>(bm + W);
  int32_t *cnt = pre + W;
  int32_t *sbase = cnt + (lds_cnt ? R : 0);
  const int64_t row0 = seg_off[cbase];
  if (lds_slot) {
    for (int32_t t = lane; t < W; t += 64) bm[t] = 0u;
    __syncthreads();
    for (int64_t e = cbase + lane; e < cbase + R; e += 64) bm_set(bm, c_ci[e]);
    __syncthreads();
    // prefix popcount (single wavefront)
    int32_t per = (W + 63) / 64;
    int32_t w0 = lane * per, w1 = min(W, w0 + per);
    int32_t s = 0;
    for (int32_t w = w0; w < w1; w++) s += __popc(bm[w]);
    int32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    int32_t r = inc - s;
    for (int32_t w = w0; w < w1; w++) {
      pre[w] = r;
      r += __popc(bm[w]);
    }
  }
  if (lds_cnt)
    for (int32_t t = lane; t < R; t += 64) {
      cnt[t] = 0;
      sbase[t] = (int32_t)(seg_off[cbase + t] - row0) + (kofs ? kofs[(cbase + t) * nk1 + pass] : 0);
    }
  __syncthreads();
  int32_t *gcur = run ? run + cbase * nk1 : nullptr;   // wide rows: global cursors per (slot, pass)
  const int64_t pa0 = A.rp[i], pa1 = A.rp[i + 1];
  for (int64_t pb = pa0; pb < pa1; pb += 64) {
    const int64_t p = pb + lane;
    bool ok = false;
    int64_t qb = 0;
    int32_t nq = 0;
    uint32_t ea = 0u, kb = 0u;
    double nA = 0.0;
    if (p < pa1) {
      const int32_t k = A.ci[p];
      const int32_t kc = A.cbs[k];
      if (nks == 0 || kc == ksz.v[pass]) {
        qb = B.rp[k];
        nq = (int32_t)(B.rp[k + 1] - qb);
        ok = nq > 0;
        const int32_t ablk = A.blk ? A.blk[p] : (int32_t)p;
        nA = na ? na[ablk] : 0.0;
        ea = enc ? ((uint32_t)((A.off[ablk] - abase) * 8) | (uint32_t)((kc - 1) & 7)) : (uint32_t)ablk;
        kb = enc ? (uint32_t)((kc - 1) >> 3) : 0u;
      }
    }
    const uint64_t m = __ballot(ok);
    const int ne = __popcll(m);
    if (ok) {
      const int t = __popcll(m & ((1ull << lane) - 1ull));
      s_qb[t] = qb;
      s_na[t] = nA;
      s_nq[t] = nq;
      s_ea[t] = ea;
      s_kb[t] = kb;
    }
    __syncthreads();
    // the common case (slots and cursors in LDS) has a loop of its own, with
    // no global load besides the ring's, so the loads stay in flight
    auto walk = [&](auto fast) {
      constexpr bool FAST = decltype(fast)::value;
      chunk_walk<BEnt>(s_qb, s_nq, ne, [&](int64_t q) { return bent[q]; }, [&](int e, const BEnt &v) {
        if (na && (s_na[e] * v.nb < eps)) return;
        int32_t slot;
        int64_t pos;
        if constexpr (FAST) {
          if (!bm_test(bm, v.j)) return;
          slot = bm_slot(bm, pre, v.j);
          const int32_t at = cnt[slot];
          cnt[slot] = at + 1;
          pos = row0 + sbase[slot] + at;
        } else {
          if (lds_slot) slot = bm_test(bm, v.j) ? bm_slot(bm, pre, v.j) : -1;
          else slot = bsearch_slot(c_ci, cbase, cbase + R, v.j);
          if (slot < 0) return;
          if (lds_cnt) {
            const int32_t at = cnt[slot];
            cnt[slot] = at + 1;
            pos = row0 + sbase[slot] + at;
          } else {
            const int32_t at = atomicAdd(&gcur[slot * nk1 + pass], 1);
            pos = seg_off[cbase + slot] + (kofs ? kofs[(cbase + slot) * nk1 + pass] : 0) + at;
          }
        }
        // encoded: byte offsets of the two packed blocks, k size - 1 in their low 3 + 2 bits
        stack[pos] = make_int2((int)s_ea[e], (int)(v.eb | s_kb[e]));
      });
    };
    if (lds_slot && lds_cnt) walk(std::true_type{});
    else walk(std::false_type{});
    __syncthreads();   // the opened entries are rewritten by the next batch
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (pad4) {
    // close this k size: pad every C block's run to a multiple of 4 entries
    for (int32_t t = lane; t < R; t += 64) {
      int32_t at;
      int64_t b0;
      if (lds_cnt) {
        at = cnt[t];
        b0 = row0 + sbase[t];
      } else {
        at = atomicAdd(&gcur[t * nk1 + pass], 0);
        b0 = seg_off[cbase + t] + (kofs ? kofs[(cbase + t) * nk1 + pass] : 0);
      }
      const int32_t gm = (diag8 && A.rbs[i] <= 8 && B.cbs[c_ci[cbase + t]] <= 8) ? 7 : 3;
      const int32_t end = (at + gm) & ~gm;
      for (; at < end; at++)
        stack[b0 + at] = enc ? make_int2((int)0x80000000u, (int)0x80000000u) : make_int2(-1, -1);
    }
  }
}

// First entry of every block row whose column is at least w * wc, for
// w = 0 .. nwin (one row per workgroup; the last is the row's end).  With
// row_max, the largest number of entries of row r inside one window (in row_max[r]).
__global__ __launch_bounds__(256) void k_window_bounds(const int64_t *rp, const int32_t *ci, int32_t wc, int nwin,
                                                      int64_t *out, int32_t *row_max) {
  extern __shared__ int64_t wb[];
  const int32_t r = blockIdx.x;
  const int t = threadIdx.x, nt = blockDim.x;
  const int64_t q0 = rp[r], q1 = rp[r + 1];
  for (int w = t; w <= nwin; w += nt) wb[w] = q1;
  __syncthreads();
  for (int64_t q = q0 + t; q < q1; q += nt) {
    const int wq = ci[q] / wc;
    const int wp = (q == q0) ? -1 : ci[q - 1] / wc;
    for (int w = wp + 1; w <= wq; w++) wb[w] = q;   // windows opened by entry q
  }
  __syncthreads();
  for (int w = t; w <= nwin; w += nt) out[(int64_t)r * (nwin + 1) + w] = wb[w];
  if (row_max) {   // windows are held by the first wavefront (nwin <= 64)
    int32_t mx = 0;
    for (int w = t; w < nwin; w += nt) mx = max(mx, (int32_t)(wb[w + 1] - wb[w]));
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
    if (t == 0) row_max[r] = mx;
  }

}

// Stack generation for one (C block row i, k size, column window): the
// window holds the C blocks of row i with j in [w*wc, (w+1)*wc), and the
// products are taken from the part of each B row inside the window (the
// window bounds of op(B)'s rows).  Products go through the same ordered LDS
// cursors as above, but a C block's entries are not written one by one:
// they gather in an LDS group of four, and the fourth sends the group (32
// aligned bytes, runs being padded to groups of four) in one write; the
// last group of a run is completed with null entries at the end.  The window
// keeps the LDS cost per C block (group, cursor, run start) within budget,
// so memory sees whole 32-byte groups instead of scattered 8-byte writes.
// Without buffering (more C blocks in the window than buf_cap), entries go
// straight to memory and the runs are padded afterwards.
__global__ __launch_bounds__(64) void k_stack_fill_win(OpView A, OpView B, const int64_t *wslot, const int64_t *bwin,
                                                       int nwin, int32_t wc, const int32_t *c_ci,
                                                       const int64_t *seg_off, const int32_t *kofs, int2 *stack,
                                                       const BEnt *bent, const double *na, double eps,
                                                       int32_t buf_cap, KSizes ksz, int nks, int32_t nbr,
                                                       const int32_t *ord, int64_t per_xcd, int diag8,
                                                       const int64_t *a_base, int plain) {
  extern __shared__ uint32_t sm[];
  const RowUnit ru = row_unit(nbr, nks * nwin, per_xcd, ord);
  if (!ru.ok) return;
  const int32_t i = ru.row;
  const int64_t abase = a_base ? a_base[i] : 0;   // encoded A offsets start at row i's packed blocks
  const int pass = ru.unit / nwin, w = ru.unit - pass * nwin;
  const int lane = threadIdx.x;
  const int64_t s0 = wslot[(int64_t)i * (nwin + 1) + w], s1 = wslot[(int64_t)i * (nwin + 1) + w + 1];
  const int32_t ns = (int32_t)(s1 - s0);
  if (ns == 0) return;
  const int32_t j0 = w * wc;
  const int32_t W = (wc + 31) >> 5;
  // plain entries (block ids, every k in one pass, no padding) go straight
  // to memory: their runs do not start on groups of four
  const bool buffered = !plain && ns <= buf_cap;
  int64_t *s_qb = reinterpret_cast<int64_t *>(sm);
  double *s_na = reinterpret_cast<double *>(sm + 128);
  int32_t *s_nq = reinterpret_cast<int32_t *>(sm + 256);
  uint32_t *s_ea = sm + 320;
  uint32_t *s_kb = sm + 384;
  int2 *buf = reinterpret_cast<int2 *>(sm + STACK_LDS_HEAD / 4);   // a group of 4 per C block
  uint32_t *bm = reinterpret_cast<uint32_t *>(buf + (buffered ? 4 * ns : 0));
  int32_t *pre = reinterpret_cast<int32_t *>(bm + W);
  int32_t *cnt = pre + W;
  int32_t *sbase = cnt + ns;
  const int64_t g0 = seg_off[s0];
  for (int32_t t = lane; t < W; t += 64) bm[t] = 0u;
  __syncthreads();
  for (int64_t c = s0 + lane; c < s1; c += 64) bm_set(bm, c_ci[c] - j0);
  __syncthreads();
  {
    const int32_t per = (W + 63) / 64;
    const int32_t w0 = lane * per, w1 = min(W, w0 + per);
    int32_t sum = 0;
    for (int32_t u = w0; u < w1; u++) sum += __popc(bm[u]);
    int32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    int32_t r = inc - sum;
    for (int32_t u = w0; u < w1; u++) {
      pre[u] = r;
      r += __popc(bm[u]);
    }
  }
  for (int32_t t = lane; t < ns; t += 64) {
    cnt[t] = 0;
    sbase[t] = (int32_t)(seg_off[s0 + t] - g0) + (plain ? 0 : kofs[(s0 + t) * nks + pass]);
  }
  __syncthreads();
  int2 *base = stack + g0;
  const int64_t pa0 = A.rp[i], pa1 = A.rp[i + 1];
  for (int64_t pb = pa0; pb < pa1; pb += 64) {
    const int64_t p = pb + lane;
    bool ok = false;
    int64_t qb = 0;
    int32_t nq = 0;
    uint32_t ea = 0u, kb = 0u;
    double nA = 0.0;
    if (p < pa1) {
      const int32_t k = A.ci[p];
      const int32_t kc = A.cbs[k];
      if (plain || kc == ksz.v[pass]) {
        const int64_t *bw = bwin + (int64_t)k * (nwin + 1) + w;
        qb = bw[0];
        nq = (int32_t)(bw[1] - qb);
        ok = nq > 0;
        const int32_t ablk = A.blk ? A.blk[p] : (int32_t)p;
        nA = na ? na[ablk] : 0.0;
        if (plain) {
          ea = (uint32_t)ablk;
        } else {
          ea = (uint32_t)((A.off[ablk] - abase) * 8) | (uint32_t)((kc - 1) & 7);
          kb = (uint32_t)((kc - 1) >> 3);
        }
      }
    }
    const uint64_t m = __ballot(ok);
    const int ne = __popcll(m);
    if (ok) {
      const int t = __popcll(m & ((1ull << lane) - 1ull));
      s_qb[t] = qb;
      s_na[t] = nA;
      s_nq[t] = nq;
      s_ea[t] = ea;
      s_kb[t] = kb;
    }
    __syncthreads();
    // buffered and direct writing are separate loops: a store common to both
    // would be merged into one generic (flat) store, which the compiler
    // then orders against every load in flight
    auto walk = [&](auto buffered_t) {
      constexpr bool BUF = decltype(buffered_t)::value;
      chunk_walk<BEnt, 16>(s_qb, s_nq, ne, [&](int64_t q) { return bent[q]; }, [&](int e, const BEnt &v) {
        if (na && (s_na[e] * v.nb < eps)) return;
        const int32_t jj = v.j - j0;
        if (!bm_test(bm, jj)) return;   // only under retain_sparsity
        const int32_t slot = bm_slot(bm, pre, jj);
        const int32_t at = cnt[slot];
        cnt[slot] = at + 1;
        // encoded: byte offsets of the two packed blocks, k size - 1 in their low 3 + 2 bits
        const int2 ent = make_int2((int)s_ea[e], (int)(v.eb | s_kb[e]));
        if constexpr (BUF) {
          buf[slot * 4 + (at & 3)] = ent;
          if ((at & 3) == 3) {   // group complete: its 32 bytes in one go
            const int4 *src = reinterpret_cast<const int4 *>(buf + slot * 4);
            int4 *dst = reinterpret_cast<int4 *>(base + sbase[slot] + (at - 3));
            dst[0] = src[0];
            dst[1] = src[1];
          }
        } else {
          base[sbase[slot] + at] = ent;
        }
      });
    };
    if (buffered) walk(std::true_type{});
    else walk(std::false_type{});
    __syncthreads();   // the opened entries are rewritten by the next batch
  }
  if (plain) return;   // runs hold exactly their products
  // close every run of this k size: the groups of four from the one holding
  // the last entry up to the padded end (a multiple of four, of eight for
  // the diagonal-packed variant's blocks), null entries past the last
  const int nul = (int)0x80000000u;
  const bool m8 = diag8 && A.rbs[i] <= 8;
  for (int32_t t = lane; t < ns; t += 64) {
    const int32_t at = cnt[t];
    const int32_t gm = (m8 && B.cbs[c_ci[s0 + t]] <= 8) ? 7 : 3;
    const int32_t end = (at + gm) & ~gm;
    for (int32_t gs = at & ~3; gs < end; gs += 4) {
      int2 *g = base + sbase[t] + gs;
      if (buffered) {
        int2 x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = gs + u < at ? buf[t * 4 + u] : make_int2(nul, nul);
        int4 *dst = reinterpret_cast<int4 *>(g);
        dst[0] = make_int4(x[0].x, x[0].y, x[1].x, x[1].y);
        dst[1] = make_int4(x[2].x, x[2].y, x[3].x, x[3].y);
      } else {
        for (int u = max(at - gs, 0); u < 4; u++) g[u] = make_int2(nul, nul);
      }
    }
  }
}

// Whether the on-the-fly filter decision of any candidate product changes
// between two sets of block norms (na0, nb0: those a plan was built with;
// na1, nb1: the current ones): for every row i of op(A), entry (i, k) and
// entry (k, j) of op(B), kept iff !(||A_ik|| ||B_kj|| < eps) under each
// set, the same expression as the stack generator's.  One workgroup per
// row; a difference sets *flag, after which remaining rows return at once.
__global__ __launch_bounds__(256) void k_decisions_differ(OpView A, OpView B, int32_t nbr, const double *na0,
                                                          const double *nb0, const double *na1, const double *nb1,
                                                          double eps, int32_t *flag) {
  const int32_t i = blockIdx.x;
  if (i >= nbr || __atomic_load_n(flag, __ATOMIC_RELAXED)) return;   // uniform over the workgroup
  for (int64_t pa = A.rp[i]; pa < A.rp[i + 1]; pa++) {
    const int32_t k = A.ci[pa];
    const int32_t a = A.blk ? A.blk[pa] : (int32_t)pa;
    const double x0 = na0[a], x1 = na1[a];
    int diff = 0;
    for (int64_t q = B.rp[k] + threadIdx.x; q < B.rp[k + 1]; q += blockDim.x) {
      const int32_t b = B.blk ? B.blk[q] : (int32_t)q;
      const bool keep0 = !(x0 * nb0[b] < eps), keep1 = !(x1 * nb1[b] < eps);
      diff |= keep0 != keep1;
    }
    if (__syncthreads_or(diff)) {
      if (threadIdx.x == 0) atomicOr(flag, 1);
      return;
    }
  }
}

}  // namespace

void decisions_differ(const OpIndex &a, const OpIndex &b, const double *na0, const double *nb0, const double *na1,
                      const double *nb1, double eps, int32_t *flag, hipStream_t s) {
  if (a.nbr == 0) return;
  hipLaunchKernelGGL(k_decisions_differ, dim3((unsigned)a.nbr), dim3(256), 0, s, view(a), view(b), a.nbr, na0, nb0,
                     na1, nb1, eps, flag);
  HIPCHECK(hipGetLastError());
}

size_t symbolic_bits_words(int32_t nbr, int32_t nbc) {
  const int64_t words_total = ((int64_t)nbc + 31) >> 5;
  if (words_total == 0 || words_total > MAX_WORDS) return 0;
  const size_t n = (size_t)nbr * (size_t)words_total;
  return n * 4 <= ((size_t)256 << 20) ? n : 0;
}

void symbolic_count(const SymArgs &g, int64_t *row_nnz, int32_t *max_row, hipStream_t s) {
  int32_t nbr = g.a->nbr;
  if (nbr == 0) return;
  int32_t words_total = (g.nbc + 31) >> 5;
  int32_t W = std::min(words_total, MAX_WORDS);
  if (W == 0) {
    HIPCHECK(hipMemsetAsync(row_nnz, 0, sizeof(int64_t) * nbr, s));
    return;
  }
  const int64_t px = row_units_per_xcd(nbr, 1);
  hipLaunchKernelGGL(k_sym_count, dim3((unsigned)(px * 8)), dim3(SYM_THREADS), W * sizeof(uint32_t), s, view(*g.a),
                     view(*g.b), g.cold_rp, g.cold_ci, g.use_cold ? 1 : 0, g.nbc, row_nnz, max_row, nbr, g.ord, px,
                     words_total <= MAX_WORDS ? g.bits : nullptr);
  HIPCHECK(hipGetLastError());
}

void symbolic_fill(const FillArgs &f, hipStream_t s) {
  int32_t nbr = f.sym.a->nbr;
  if (nbr == 0) return;
  int32_t words_total = (f.sym.nbc + 31) >> 5;
  int32_t W = std::min(words_total, MAX_WORDS);
  if (W == 0) W = 1;
  KSizes ks;
  const int nkp = f.pad4 ? (int)f.ksizes.size() : 0;
  for (int t = 0; t < nkp; t++) ks.v[t] = f.ksizes[t];
  int32_t cap = (int32_t)std::min<int64_t>((int64_t)f.max_row * std::max(nkp, 1), SYM_CNT_CAP);
  size_t lds = (size_t)W * 8 + (size_t)std::max(cap, 1) * 4;
  if (lds + sizeof(AOpen) * (SYM_THREADS / 64) + 1024 > 65536)
    HIPCHECK(hipFuncSetAttribute((const void *)k_sym_fill, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t px = row_units_per_xcd(nbr, 1);
  hipLaunchKernelGGL(k_sym_fill, dim3((unsigned)(px * 8)), dim3(SYM_THREADS), lds, s, view(*f.sym.a), view(*f.sym.b),
                     f.sym.cold_rp, f.sym.cold_ci, f.sym.use_cold ? 1 : 0, f.sym.retain ? 1 : 0, f.sym.nbc,
                     f.c_rp, f.c_ci, f.c_row, f.c_size, f.c_cnt, f.c_kflops, f.row_cand, f.row_real,
                     reinterpret_cast<const BEnt *>(f.bent), f.na, f.eps, cap, ks, nkp, f.cnt_g,
                     nkp > 0 ? f.kofs : nullptr, nbr, f.sym.ord, px,
                     (words_total <= MAX_WORDS && !f.sym.retain) ? f.sym.bits : nullptr,
                     (f.diag8 && nkp > 0) ? 1 : 0, reinterpret_cast<unsigned long long *>(f.margin));
  HIPCHECK(hipGetLastError());
}

void old_block_map(const int64_t *cold_rp, const int32_t *cold_ci, int32_t nbr, const int64_t *c_rp,
                   const int32_t *c_ci, int32_t *old_blk, hipStream_t s) {
  if (nbr == 0) return;
  hipLaunchKernelGGL(k_old_map, dim3(nbr), dim3(256), 0, s, cold_rp, cold_ci, c_rp, c_ci, old_blk);
  HIPCHECK(hipGetLastError());
}

void product_records(const OpIndex &b, const double *nb, const int64_t *b_poff, const int64_t *b_base, int4 *out,
                     hipStream_t s) {
  if (b.nnzb == 0) return;
  OpView vb = view(b);
  if (b_poff) vb.off = b_poff;   // encoded entries: offsets into the packed copy of op(B)
  hipLaunchKernelGGL(k_product_records, dim3((unsigned)std::min<int64_t>((b.nnzb + 255) / 256, 65536)), dim3(256), 0, s,
                     vb, b.nnzb, nb, b_poff ? 1 : 0, b_poff ? b_base : nullptr, reinterpret_cast<BEnt *>(out));
  HIPCHECK(hipGetLastError());
}

StackWindows stack_windows(int32_t nbc, int32_t max_row, int nks) {
  StackWindows sw;
  const int32_t words_total = (nbc + 31) >> 5;
  if (nks < 1 || nks > MAX_KSIZES || words_total == 0 || words_total > MAX_WORDS || max_row < 1) return sw;
  // 32 bytes of LDS per C block of a window for its group of four entries:
  // windows narrow enough that the widest row's share fits
  int nwin = (int)std::min<int64_t>(16, std::max<int64_t>(1, ((int64_t)max_row * 32 + STACK_BUF_BYTES - 1) /
                                                                 STACK_BUF_BYTES));
  const int32_t wc = (int32_t)((((int64_t)nbc + nwin - 1) / nwin + 31) & ~(int64_t)31);
  nwin = (int)(((int64_t)nbc + wc - 1) / wc);
  // the kernel's LDS for a window of ns C blocks (ns <= min(max_row, wc)):
  // the opened A entries, groups of four entries (up to the buffer), the
  // window's bitmap and prefix words, a cursor and a run start per C block;
  // wider windows go to the unwindowed generator
  const int64_t ns = std::min<int64_t>(max_row, wc);
  const int64_t lds = (int64_t)STACK_LDS_HEAD + std::min<int64_t>(ns, STACK_BUF_BYTES / 32) * 32 +
                      (int64_t)((wc + 31) >> 5) * 8 + ns * 8;
  if (lds > 65536) return sw;
  sw.nwin = nwin;
  sw.wc = wc;
  return sw;
}

void window_bounds(const int64_t *rp, const int32_t *ci, int32_t nrows, const StackWindows &sw, int64_t *out,
                   int32_t *row_max, hipStream_t s) {
  if (nrows == 0 || sw.nwin < 1) return;
  hipLaunchKernelGGL(k_window_bounds, dim3(nrows), dim3(256), sizeof(int64_t) * (sw.nwin + 1), s, rp, ci, sw.wc,
                     sw.nwin, out, row_max);
  HIPCHECK(hipGetLastError());
}

void stack_fill(const StackArgs &g, int32_t *run, hipStream_t s) {
  if (g.nbr == 0) return;
  int32_t words_total = (g.nbc + 31) >> 5;
  int32_t W = std::min(words_total, MAX_WORDS);
  if (W == 0) W = 1;
  int32_t cap = std::min(g.max_row, CNT_CAP / 2);
  // opened A entries, bitmap + prefix, cursors + run starts
  size_t lds = STACK_LDS_HEAD + (size_t)W * 8 + (size_t)std::max(cap, 1) * 8;
  KSizes ks;
  int nks = g.pad4 ? (int)g.ksizes.size() : 0;
  if (nks > MAX_KSIZES) nks = 0;
  for (int t = 0; t < nks; t++) ks.v[t] = g.ksizes[t];
  OpView va = view(*g.a), vb = view(*g.b);
  if (g.encode) {   // entries carry offsets into the packed operand copies
    va.off = g.a_poff;
  }
  const BEnt *bent = reinterpret_cast<const BEnt *>(g.bent);
  // windowed: encoded entries in padded k-size runs (quad path), or plain
  // block ids with every k in one pass (tile and pointer paths)
  const bool plain = !g.pad4 && !g.encode;
  if (g.win.nwin > 0 && ((g.pad4 && g.encode && nks > 0) || plain)) {
    const int32_t buf_cap = (int32_t)(STACK_BUF_BYTES / 32);
    const int32_t ns = std::max(g.max_ns, 1);
    const int32_t Ww = (g.win.wc + 31) >> 5;
    const size_t lw = STACK_LDS_HEAD + (size_t)std::min(ns, buf_cap) * 32 + (size_t)Ww * 8 + (size_t)ns * 8;
    if (lw > 65536)
      HIPCHECK(hipFuncSetAttribute((const void *)k_stack_fill_win, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lw));
    const int nkw = plain ? 1 : nks;   // k-size passes per row (plain: one for every k)
    const int64_t px = row_units_per_xcd(g.nbr, nkw * g.win.nwin);
    hipLaunchKernelGGL(k_stack_fill_win, dim3((unsigned)(px * 8)), dim3(64), lw, s, va, vb, g.wslot, g.bwin,
                       g.win.nwin, g.win.wc, g.c_ci, g.seg_off, plain ? nullptr : g.kofs, g.stack, bent, g.na,
                       g.eps, buf_cap, ks, nkw, g.nbr, g.ord, px, (g.diag8 && !plain) ? 1 : 0,
                       plain ? nullptr : g.a_base, plain ? 1 : 0);
    HIPCHECK(hipGetLastError());
    return;
  }
  const int64_t px = row_units_per_xcd(g.nbr, std::max(nks, 1));
  hipLaunchKernelGGL(k_stack_fill, dim3((unsigned)(px * 8)), dim3(64), lds, s, va, vb, g.nbc, g.c_rp, g.c_ci,
                     g.seg_off, nks > 0 ? g.kofs : nullptr, g.stack, bent, g.na, g.eps, cap, run, ks, nks,
                     g.pad4 ? 1 : 0, g.encode ? 1 : 0, g.nbr, g.ord, px, g.diag8 ? 1 : 0, g.encode ? g.a_base : nullptr);
  HIPCHECK(hipGetLastError());
}

}  // namespace bsmm
