// index_kernels.hip -- device-wide scans, the block-index transpose (op = T),
// block Frobenius norms and the compaction used by the post-multiply filter.
#include "internal.h"

namespace bsmm {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Inclusive scan over a 64-wide wavefront.
__device__ inline int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive prefix of `v` over the 256 threads of the block; total in *tot.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *tot) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v, lane);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int64_t base = 0, all = 0;
  for (int t = 0; t < SCAN_THREADS / 64; t++) {
    if (t < w) base += sh[t];
    all += sh[t];
  }
  __syncthreads();
  *tot = all;
  return base + inc - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_sums(const T *in, int64_t n, int64_t *sums) {
  __shared__ int64_t sh[SCAN_THREADS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; t++)
    if (base + t < n) s += (int64_t)in[base + t];
  int64_t tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_scan(const T *in, int64_t n, const int64_t *tile_base,
                                                            int64_t *out) {
  __shared__ int64_t sh[SCAN_THREADS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; t++) {
    v[t] = (base + t < n) ? (int64_t)in[base + t] : 0;
    s += v[t];
  }
  int64_t tot;
  int64_t run = block_excl_scan(s, sh, &tot) + (tile_base ? tile_base[blockIdx.x] : 0);
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; t++) {
    if (base + t < n) out[base + t] = run;
    run += v[t];
  }
  // the block holding element n-1 (or block 0 when n == 0) writes the total
  int64_t last_blk = n > 0 ? (n - 1) / SCAN_TILE : 0;
  if ((int64_t)blockIdx.x == last_blk && threadIdx.x == SCAN_THREADS - 1) {
    out[n] = (tile_base ? tile_base[blockIdx.x] : 0) + tot;
  }
}

template <typename T>
void scan_impl(Allocator &al, const T *in, int64_t *out, int64_t n, hipStream_t s) {
  int64_t tiles = n > 0 ? (n + SCAN_TILE - 1) / SCAN_TILE : 1;
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(SCAN_THREADS), 0, s, in, n, (const int64_t *)nullptr, out);
    HIPCHECK(hipGetLastError());
    return;
  }
  DBuf<int64_t> sums(al, tiles), base(al, tiles + 1);
  hipLaunchKernelGGL(k_tile_sums<T>, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, n, sums.p);
  HIPCHECK(hipGetLastError());
  scan_impl<int64_t>(al, sums.p, base.p, tiles, s);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, n, (const int64_t *)base.p, out);
  HIPCHECK(hipGetLastError());
}

// ------------------------------------------------------------- transpose
// Rows are processed in chunks of R rows.  cc[c*nbc + j] first counts the
// blocks of column j inside chunk c, then (after a scan down the chunks)
// holds where chunk c starts writing inside new row j.  Chunks fill in
// parallel; inside a chunk one wavefront walks its rows in order, so every
// new row ends up sorted by old row.

__global__ void k_tr_count(const int64_t *rp, const int32_t *ci, int32_t nbr, int32_t rows_per_chunk,
                           int32_t nbc, int32_t *cc) {
  int32_t chunk = blockIdx.x;
  int32_t r0 = chunk * rows_per_chunk, r1 = min(nbr, r0 + rows_per_chunk);
  if (r0 >= r1) return;
  int64_t p0 = rp[r0], p1 = rp[r1];
  int32_t *row = cc + (int64_t)chunk * nbc;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) atomicAdd(&row[ci[p]], 1);
}

__global__ void k_tr_colscan(int32_t *cc, int32_t nchunks, int32_t nbc, int64_t *colcount) {
  int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nbc) return;
  int32_t run = 0;
  for (int32_t c = 0; c < nchunks; c++) {
    int64_t idx = (int64_t)c * nbc + j;
    int32_t v = cc[idx];
    cc[idx] = run;
    run += v;
  }
  colcount[j] = run;
}

__global__ __launch_bounds__(64) void k_tr_fill(const int64_t *rp, const int32_t *ci, int32_t nbr,
                                                int32_t rows_per_chunk, int32_t nbc, int32_t *cc,
                                                const int64_t *rpT, int32_t *ciT, int32_t *blkT) {
  int32_t chunk = blockIdx.x;
  int32_t r0 = chunk * rows_per_chunk, r1 = min(nbr, r0 + rows_per_chunk);
  int32_t *row = cc + (int64_t)chunk * nbc;
  for (int32_t i = r0; i < r1; i++) {
    for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 64) {
      int32_t j = ci[p];
      // columns are distinct inside one old row; the atomic keeps successive
      // rows of this wavefront ordered on the same counter
      int32_t slot = atomicAdd(&row[j], 1);
      int64_t q = rpT[j] + slot;
      ciT[q] = i;
      blkT[q] = (int32_t)p;
    }
  }
}

// ------------------------------------------------------------------ norms
// 16 lanes per block, U blocks per lane group in flight: the group reads the
// U blocks' offsets together, then issues one load per block per step
// (indices clamped into the block, so there are no branches between the
// loads) before it accumulates.  Each lane sums its elements in ascending
// order and the 16 partial sums combine in a fixed tree: the result does not
// depend on the launch.
template <int U>
__global__ __launch_bounds__(256) void k_block_norms(const int64_t *off, const double *v, int64_t nnzb,
                                                     double *out) {
  constexpr int G = 16;
  const int lane = threadIdx.x % G;
  const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t b0 = grp * U; b0 < nnzb; b0 += ngrp * U) {
    int64_t o0[U], len[U];
    int64_t lmax = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t b = min(b0 + u, nnzb - 1);
      o0[u] = off[b];
      len[u] = (b0 + u < nnzb) ? off[b + 1] - o0[u] : 0;
      lmax = max(lmax, len[u]);
    }
    double s[U];
#pragma unroll
    for (int u = 0; u < U; u++) s[u] = 0.0;
    // unrolled: several iterations' loads in flight, the sums still taken in
    // the order of d
#pragma unroll 4
    for (int64_t d = lane; d < lmax; d += G) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; u++) x[u] = v[o0[u] + min(d, max(len[u] - 1, (int64_t)0))];
#pragma unroll
      for (int u = 0; u < U; u++)
        if (d < len[u]) s[u] = fma(x[u], x[u], s[u]);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int dd = G / 2; dd >= 1; dd >>= 1) s[u] += __shfl_xor(s[u], dd, G);
      if (lane == 0 && b0 + u < nnzb) out[b0 + u] = sqrt(s[u]);
    }
  }
}

// ------------------------------------------------------------- compaction
__global__ void k_keep_flags(const double *norm, double eps, int64_t n, int32_t *keep) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) keep[c] = (norm[c] < eps) ? 0 : 1;   // dropped iff norm < eps
}

__global__ void k_new_rowptr(const int64_t *rp, int32_t nbr, const int64_t *rank, int64_t *new_rp) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= nbr) new_rp[i] = rank[rp[i]];
}

__global__ void k_compact_index(const int64_t *rp, int32_t nbr, const int32_t *ci, const int64_t *rank,
                                const int32_t *rbs, const int32_t *cbs, int32_t *new_ci, int64_t *new_size) {
  int32_t i = blockIdx.x;
  int64_t m = rbs[i];
  for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += blockDim.x) {
    int64_t r = rank[p];
    if (rank[p + 1] != r) {
      int32_t j = ci[p];
      new_ci[r] = j;
      new_size[r] = m * cbs[j];
    }
  }
}

__global__ __launch_bounds__(256) void k_compact_values(const int64_t *rank, int64_t nnzb, const int64_t *off,
                                                        const double *v, const int64_t *new_off, double *nv) {
  int lane = threadIdx.x & 63;
  int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t b = w; b < nnzb; b += nw) {
    int64_t r = rank[b];
    if (rank[b + 1] == r) continue;
    int64_t o0 = off[b], len = off[b + 1] - o0, d0 = new_off[r];
    for (int64_t e = lane; e < len; e += 64) nv[d0 + e] = v[o0 + e];
  }
}

int grid_for(int64_t items, int per_block, int cap = 65536) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

namespace {
// Work list sorted by (tile of the row in the locality order, rank of the
// column).  A tile of tile_rows rows is split into subtiles of 16 rows, one
// workgroup each.  Pass 1 counts the subtile's C blocks per column in LDS
// and stores the counts under the key (tile, column rank, subtile); an
// exclusive scan over the keys gives every (tile, column, subtile) its first
// place; pass 2 places the subtile's blocks through LDS cursors.  Blocks of
// one column and subtile land in any order: the order of work items changes
// no result (each C block is summed by one wavefront in its own fixed order).
constexpr int32_t WL_SUB = 16;

__global__ __launch_bounds__(256) void k_wl_count(const int32_t *ord, const int32_t *crank, const int64_t *c_rp,
                                                  const int32_t *c_ci, int32_t nbr, int32_t nbc, int32_t nsub,
                                                  int32_t *cnt) {
  extern __shared__ int32_t hist[];
  const int32_t g = blockIdx.x, tile = g / nsub, sub = g - tile * nsub;
  for (int32_t j = threadIdx.x; j < nbc; j += blockDim.x) hist[j] = 0;
  __syncthreads();
  for (int32_t r = g * WL_SUB; r < min(nbr, (g + 1) * WL_SUB); r++) {
    const int64_t c0 = c_rp[ord[r]], c1 = c_rp[ord[r] + 1];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
      const int32_t col = c_ci[c];
      atomicAdd(&hist[crank ? crank[col] : col], 1);
    }
  }
  __syncthreads();
  for (int32_t j = threadIdx.x; j < nbc; j += blockDim.x)
    cnt[((int64_t)tile * nbc + j) * nsub + sub] = hist[j];
}

__global__ __launch_bounds__(256) void k_wl_place(const int32_t *ord, const int32_t *crank, const int64_t *c_rp,
                                                  const int32_t *c_ci, int32_t nbr, int32_t nbc, int32_t nsub,
                                                  const int64_t *first, int32_t *c_list, int32_t *pos) {
  extern __shared__ int32_t cur[];
  const int32_t g = blockIdx.x, tile = g / nsub, sub = g - tile * nsub;
  for (int32_t j = threadIdx.x; j < nbc; j += blockDim.x)
    cur[j] = (int32_t)first[((int64_t)tile * nbc + j) * nsub + sub];
  __syncthreads();
  for (int32_t r = g * WL_SUB; r < min(nbr, (g + 1) * WL_SUB); r++) {
    const int64_t c0 = c_rp[ord[r]], c1 = c_rp[ord[r] + 1];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
      const int32_t col = c_ci[c];
      const int32_t at = atomicAdd(&cur[crank ? crank[col] : col], 1);
      c_list[at] = (int32_t)c;
      if (pos) pos[c] = at;
    }
  }
}
}  // namespace

void build_work_list_sorted(Allocator &al, const int32_t *ord, const int32_t *crank, const int64_t *c_rp,
                            const int32_t *c_ci, int64_t nnzb_c, int32_t nbr, int32_t nbc, int32_t tile_rows,
                            int32_t *c_list, int32_t *pos, hipStream_t s) {
  if (nnzb_c <= 0 || nbr <= 0) return;
  const int32_t nsub = tile_rows / WL_SUB;
  const int32_t ngroups = (nbr + WL_SUB - 1) / WL_SUB;
  const int64_t ntile = (ngroups + nsub - 1) / nsub;
  const int64_t nkeys = ntile * nbc * nsub;
  DBuf<int32_t> cnt(al, (size_t)nkeys);
  DBuf<int64_t> first(al, (size_t)nkeys + 1);
  const size_t lds = sizeof(int32_t) * (size_t)nbc;
  if (lds > 65536) {
    HIPCHECK(hipFuncSetAttribute((const void *)k_wl_count, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HIPCHECK(hipFuncSetAttribute((const void *)k_wl_place, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  // every (tile, subtile) slot writes its counts; those past the last row write zeros
  hipLaunchKernelGGL(k_wl_count, dim3((unsigned)(ntile * nsub)), dim3(256), lds, s, ord, crank, c_rp, c_ci, nbr, nbc,
                     nsub, cnt.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i32(al, cnt.p, first.p, nkeys, s);
  hipLaunchKernelGGL(k_wl_place, dim3(ngroups), dim3(256), lds, s, ord, crank, c_rp, c_ci, nbr, nbc, nsub, first.p,
                     c_list, pos);
  HIPCHECK(hipGetLastError());
}

namespace {
// Work-item descriptors from the C blocks in storage order (contiguous
// reads), each 32-byte record written at its place in the work list.
__global__ __launch_bounds__(256) void k_desc_by_block(int64_t n, const int32_t *pos, const int32_t *c_row,
                                                       const int32_t *c_ci, const int32_t *rbs, const int32_t *cbs,
                                                       const int64_t *seg, const int64_t *c_off, DescBases bases,
                                                       BlkDesc *desc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  BlkDesc d;
  d.c = (int32_t)c;
  d.mn = rbs[c_row[c]] | (cbs[c_ci[c]] << 16);
  d.s0 = seg[c];
  d.ns = (int32_t)(seg[c + 1] - d.s0);
  d.co = c_off[c];
  d.pad = 0;
  desc[pos[c]] = d;
  if (bases.out) bases.out[pos[c]] = UnitBases{bases.a[c_row[c]], bases.b[c_ci[c]]};
}
}  // namespace

void build_desc_by_block(int64_t n, const int32_t *pos, const int32_t *c_row, const int32_t *c_ci, const int32_t *rbs,
                         const int32_t *cbs, const int64_t *seg, const int64_t *c_off, DescBases bases,
                         BlkDesc *desc, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_desc_by_block, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, pos, c_row, c_ci, rbs,
                     cbs, seg, c_off, bases, desc);
  HIPCHECK(hipGetLastError());
}

void exclusive_scan_i64(Allocator &al, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  scan_impl<int64_t>(al, in, out, n, s);
}
void exclusive_scan_i32(Allocator &al, const int32_t *in, int64_t *out, int64_t n, hipStream_t s) {
  scan_impl<int32_t>(al, in, out, n, s);
}

void transpose_index(Allocator &al, const bsmm_mat_s &x, OpIndex &op, hipStream_t s) {
  int32_t nbr = x.nbr, nbc = x.nbc;
  int64_t nnzb = x.nnzb;
  op.nbr = nbc;
  op.nbc = nbr;
  op.nnzb = nnzb;
  op.trans = true;
  op.own_rp = DBuf<int64_t>(al, (size_t)nbc + 1);
  op.own_ci = DBuf<int32_t>(al, nnzb > 0 ? nnzb : 1);
  op.own_blk = DBuf<int32_t>(al, nnzb > 0 ? nnzb : 1);
  if (nbr == 0 || nbc == 0 || nnzb == 0) {
    HIPCHECK(hipMemsetAsync(op.own_rp.p, 0, sizeof(int64_t) * ((size_t)nbc + 1), s));
  } else {
    int64_t cells = (int64_t)nbr * nbc;
    int32_t rpc = (int32_t)std::max<int64_t>(16, (cells + (1 << 24) - 1) >> 24);
    int32_t nch = (nbr + rpc - 1) / rpc;
    DBuf<int32_t> cc(al, (size_t)nch * nbc);
    DBuf<int64_t> colcount(al, nbc);
    HIPCHECK(hipMemsetAsync(cc.p, 0, sizeof(int32_t) * (size_t)nch * nbc, s));
    hipLaunchKernelGGL(k_tr_count, dim3(nch), dim3(256), 0, s, x.d_row_ptr, x.d_col_idx, nbr, rpc, nbc, cc.p);
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tr_colscan, dim3((nbc + 255) / 256), dim3(256), 0, s, cc.p, nch, nbc, colcount.p);
    HIPCHECK(hipGetLastError());
    exclusive_scan_i64(al, colcount.p, op.own_rp.p, nbc, s);
    hipLaunchKernelGGL(k_tr_fill, dim3(nch), dim3(64), 0, s, x.d_row_ptr, x.d_col_idx, nbr, rpc, nbc, cc.p,
                       (const int64_t *)op.own_rp.p, op.own_ci.p, op.own_blk.p);
    HIPCHECK(hipGetLastError());
  }
  op.row_ptr = op.own_rp.p;
  op.col_idx = op.own_ci.p;
  op.blk = op.own_blk.p;
}

namespace {
// One workgroup: out[0..3] = *at[0..3], out[4..6] = sums of the three
// arrays over n entries, out[7] = the largest entry of the max array (0 for
// a null pointer).  Integer sums and maxima: the result does not depend on
// the order.
__global__ __launch_bounds__(1024) void k_plan_totals(PlanTotals T, int64_t *out) {
  __shared__ int64_t red[4][16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  int64_t acc[4] = {0, 0, 0, 0};
  for (int64_t i = t; i < T.n; i += blockDim.x)
#pragma unroll
    for (int u = 0; u < 3; u++) acc[u] += T.sum[u][i];
  for (int64_t i = t; i < T.nmx; i += blockDim.x)
    acc[3] = max(acc[3], T.mx64 ? T.mx64[i] : (int64_t)T.mx32[i]);
#pragma unroll
  for (int u = 0; u < 4; u++) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const int64_t o = __shfl_xor(acc[u], d, 64);
      acc[u] = u < 3 ? acc[u] + o : max(acc[u], o);
    }
    if (lane == 0) red[u][wv] = acc[u];
  }
  __syncthreads();
  if (t < 4) {
    int64_t v = 0;
    for (int w = 0; w < nw; w++) v = t < 3 ? v + red[t][w] : max(v, red[t][w]);
    out[t < 3 ? 4 + t : 7] = v;
  } else if (t >= 8 && t < 12) {
    out[t - 8] = T.at[t - 8] ? *T.at[t - 8] : 0;
  }
}
}  // namespace

void plan_totals(const PlanTotals &T, int64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_totals, dim3(1), dim3(1024), 0, s, T, out);
  HIPCHECK(hipGetLastError());
}

void block_norms(const bsmm_mat_s &x, double *norms, hipStream_t s) {
  if (x.nnzb == 0) return;
  constexpr int U = 4;
  const int64_t groups = (x.nnzb + U - 1) / U;
  hipLaunchKernelGGL(k_block_norms<U>, dim3(grid_for(groups * 16, 256)), dim3(256), 0, s, x.d_blk_off, x.d_values,
                     x.nnzb, norms);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------- identity / residual
namespace {

// Values of the block-diagonal identity: block i (s_i x s_i) at off[i].
__global__ __launch_bounds__(256) void k_sequence(int32_t *out, int32_t n) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = t;
}

__global__ void k_identity_values(const int32_t *sizes, const int64_t *off, int32_t n, double *v) {
  const int32_t i = blockIdx.x;
  if (i >= n) return;
  const int sz = sizes[i];
  for (int e = threadIdx.x; e < sz * sz; e += blockDim.x) v[off[i] + e] = (e % sz == e / sz) ? 1.0 : 0.0;
}

// Per block row i: sum over its stored blocks of ||X_ij - shift * delta_ij I||_F^2
// (a block row with no diagonal block contributes shift^2 * s_i for it).
__global__ __launch_bounds__(64) void k_shift_dist_rows(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                       const int64_t *off, const double *v, double shift,
                                                       double *row_out) {
  const int32_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int sz = rbs[i];
  double acc = 0.0;
  bool has_diag = false;
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const bool diag = ci[p] == i;
    has_diag |= diag;
    const int64_t o0 = off[p], o1 = off[p + 1];
    for (int64_t e = o0 + lane; e < o1; e += 64) {
      double x = v[e];
      const int64_t t = e - o0;
      if (diag && (t % sz) == (t / sz)) x -= shift;
      acc = fma(x, x, acc);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane == 0) row_out[i] = acc + (has_diag ? 0.0 : shift * shift * (double)sz);
}

}  // namespace

namespace {

// flag[0] stays 0 while x[t] == y[t] for every t < n.
template <typename T>
__global__ void k_differs(const T *x, const T *y, int64_t n, int32_t *flag) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    if (x[t] != y[t]) {
      atomicOr(flag, 1);
      return;
    }
}

// Bounds of the ratios now[t] / then[t] over t < n (both non-negative):
// atomic min into out[0], max into out[1] on the bit patterns (non-negative
// doubles order like them).  Equal values give 1 (also 0 == 0); a ratio that
// is not finite (then == 0 < now, or a NaN) forces the bounds to 0 and +inf.
__global__ void k_ratio_bounds(const double *then, const double *now, int64_t n, unsigned long long *out) {
  double lo = INFINITY, hi = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double a = then[t], b = now[t];
    double r;
    if (a == b) r = 1.0;
    else if (a > 0.0 && b >= 0.0 && b < INFINITY) r = b / a;
    else r = NAN;
    if (r == r && r < INFINITY) {
      lo = fmin(lo, r);
      hi = fmax(hi, r);
    } else {
      lo = 0.0;
      hi = INFINITY;
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, d, 64));
    hi = fmax(hi, __shfl_xor(hi, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&out[0], (unsigned long long)__double_as_longlong(lo));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(hi));
  }
}

__global__ void k_set_u64(unsigned long long *p, int n, unsigned long long a, unsigned long long b) {
  const int t = threadIdx.x;
  if (t < n) p[t] = (t & 1) ? b : a;
}

}  // namespace

void differs_i64(const int64_t *x, const int64_t *y, int64_t n, int32_t *flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_differs<int64_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, y, n, flag);
  HIPCHECK(hipGetLastError());
}

void differs_i32(const int32_t *x, const int32_t *y, int64_t n, int32_t *flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_differs<int32_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, y, n, flag);
  HIPCHECK(hipGetLastError());
}

void set_pairs(double *p, int n, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long *>(p), n,
                     (unsigned long long)__builtin_bit_cast(uint64_t, a), (unsigned long long)__builtin_bit_cast(uint64_t, b));
  HIPCHECK(hipGetLastError());
}

void ratio_bounds(const double *then, const double *now, int64_t n, double *out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ratio_bounds, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, then, now, n,
                     reinterpret_cast<unsigned long long *>(out));
  HIPCHECK(hipGetLastError());
}

void identity_values(const int32_t *d_sizes, const int64_t *d_off, int32_t n, double *values, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_identity_values, dim3(n), dim3(256), 0, s, d_sizes, d_off, n, values);
  HIPCHECK(hipGetLastError());
}

void fill_sequence(int32_t *out, int32_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sequence, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n);
  HIPCHECK(hipGetLastError());
}

void shift_dist_rows(const bsmm_mat_s &x, double shift, double *row_out, hipStream_t s) {
  if (x.nbr == 0) return;
  hipLaunchKernelGGL(k_shift_dist_rows, dim3(x.nbr), dim3(64), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_blk_off,
                     x.d_values, shift, row_out);
  HIPCHECK(hipGetLastError());
}

int64_t count_kept(Allocator &al, const CompactArgs &c, int32_t *keep_tmp, int64_t *pinned, hipStream_t s,
                   DBuf<int64_t> &rank) {
  rank = DBuf<int64_t>(al, (size_t)c.nnzb + 1);
  if (c.nnzb > 0) {
    hipLaunchKernelGGL(k_keep_flags, dim3(grid_for(c.nnzb, 256, 1 << 30)), dim3(256), 0, s, c.norm, c.eps,
                       c.nnzb, keep_tmp);
    HIPCHECK(hipGetLastError());
  }
  exclusive_scan_i32(al, keep_tmp, rank.p, c.nnzb, s);
  HIPCHECK(hipMemcpyAsync(pinned, rank.p + c.nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return pinned[0];
}

void compact(Allocator &al, const CompactArgs &c, const int64_t *rank, const int32_t *d_rbs,
             const int32_t *d_cbs, int64_t *new_rp, int32_t *new_ci, int64_t *new_off, int64_t *pinned,
             double **new_values, int64_t *new_nval, hipStream_t s, double *dst) {
  hipLaunchKernelGGL(k_new_rowptr, dim3((c.nbr + 1 + 255) / 256), dim3(256), 0, s, c.rp, c.nbr, rank, new_rp);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(pinned, rank + c.nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  int64_t kept = pinned[0];
  DBuf<int64_t> sizes(al, kept > 0 ? kept : 1);
  if (c.nbr > 0) {
    hipLaunchKernelGGL(k_compact_index, dim3(c.nbr), dim3(256), 0, s, c.rp, c.nbr, c.ci, rank, d_rbs, d_cbs,
                       new_ci, sizes.p);
    HIPCHECK(hipGetLastError());
  }
  exclusive_scan_i64(al, sizes.p, new_off, kept, s);
  HIPCHECK(hipMemcpyAsync(pinned, new_off + kept, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  *new_nval = pinned[0];
  double *nv = dst ? dst : static_cast<double *>(al.alloc(sizeof(double) * (size_t)std::max<int64_t>(*new_nval, 1)));
  if (c.nnzb > 0) {
    hipLaunchKernelGGL(k_compact_values, dim3(grid_for(c.nnzb * 64, 256)), dim3(256), 0, s, rank, c.nnzb, c.off,
                       c.values, (const int64_t *)new_off, nv);
    HIPCHECK(hipGetLastError());
  }
  *new_values = nv;
}

}  // namespace bsmm
