// gemm_lowp.hip -- the block GEMM in FP32 and split-FP32 arithmetic (gfx950).
//
// Same work split as the FP64 kernel: one wavefront owns one C block, walks
// its stack segment in quads (four products of one k size, one per 16-lane
// k-group), accumulates in registers and writes C = alpha*acc + beta*C_old in
// FP64 with its norm.  The stored values, the block norms and both filter
// thresholds stay FP64; only the block products change arithmetic:
//
//   FP32  : operands rounded to FP32, V_MFMA_F32_16X16X4F32 products and FP32
//           accumulation over the whole segment, converted to FP64 at the end.
//   SPLIT : every operand x = hi + lo with hi = fp32(x), lo = fp32(x - hi);
//           per slab of four k-steps the MFMA forms the lo_a*hi_b and
//           hi_a*lo_b terms, then the hi_a*hi_b terms, in FP32 (small terms
//           first), and the slab's result is added to an FP64 accumulator,
//           so the sum over k is FP64 at a granularity of four k-steps (the
//           lo*lo term, about 2^-48 relative, is dropped).  Each slab's
//           result is still one FP32 rounding (2^-24 relative): the error
//           does not grow with K, but it is not FP64's.
//
// Matrix core: V_MFMA_F32_16X16X4F32, A[i][k] lane i+16k, B[k][j] lane j+16k,
// D[i][j] lane j+16(i/4), register i%4 (checked on the device).  C edges up
// to 32 use TM x TN tiles of 16.
//
// Operands come from packed FP32 copies in k-quad slabs: slab p of a block
// holds, for each row of op(A) (column of op(B)), its four values at
// k = 4p..4p+3 (pad zeros), so one 128-bit load brings a lane four k-steps
// and a k-group's lanes read one contiguous run.  The slab offset rides in
// the scalar offset of the buffer load; null products and padded rows or
// columns have out-of-range vector offsets and read zeros.
#include "internal.h"

namespace bsmm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr uint32_t QOOB = 0x80000000u;
constexpr int ROUND = 256;
constexpr int PF = 2;   // k-quad slabs in flight
constexpr int WPG = 1;  // wavefronts per workgroup (see the FP64 kernel)

struct LowpP {
  const float *a_hi, *a_lo, *b_hi, *b_lo;   // packed slabs (lo only for SPLIT)
  uint32_t a_bytes, b_bytes;
  const int32_t *c_list;
  const int32_t *c_row, *c_ci;
  const int32_t *rbs, *cbs;
  const int64_t *c_off, *seg;
  const int2 *stack;
  const int32_t *old_blk;
  const int64_t *old_off;
  const double *old_val;
  double *c_val;
  double *c_norm;
  double alpha, beta;
};

struct QuadLds {
  uint32_t oa[ROUND];
  uint32_t ob[ROUND];
  int32_t Kq[ROUND / 4];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void load_quads(const LowpP &P, QuadLds &ql, int64_t rb, int nr, int lane) {
  // entries: byte offsets of the two packed blocks with (k - 1) in their low
  // 3 + 2 bits; nulls are QOOB (a quad's first entry is never null)
  for (int q = lane; q < nr; q += 64) {
    const int2 e = P.stack[rb + q];
    const uint32_t oa = (uint32_t)e.x, ob = (uint32_t)e.y;
    ql.oa[q] = oa & ~7u;
    ql.ob[q] = ob & ~7u;
    if ((q & 3) == 0) ql.Kq[q >> 2] = (int)((oa & 7u) | ((ob & 7u) << 3)) + 1;
  }
  wave_sync();
}

__device__ __forceinline__ f4 load4(__amdgpu_buffer_rsrc_t r, uint32_t voff, int soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, soff, 0));
}

template <bool SPLIT, int TM, int TN>
__device__ __forceinline__ void gemm_block_lowp(const LowpP &P, int32_t c, QuadLds &ql) {
  constexpr int NA = SPLIT ? 2 : 1;   // hi (and lo) operand streams
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(P.rbs[P.c_row[c]]);
  const int n = __builtin_amdgcn_readfirstlane(P.cbs[P.c_ci[c]]);
  const int m16 = 16 * m, n16 = 16 * n;   // bytes of one k-quad slab
  const int kq = lane >> 4, l16 = lane & 15;
  int ra[TM], cb[TN];
#pragma unroll
  for (int t = 0; t < TM; t++) ra[t] = (l16 + 16 * t) < m ? l16 + 16 * t : -1;
#pragma unroll
  for (int u = 0; u < TN; u++) cb[u] = (l16 + 16 * u) < n ? l16 + 16 * u : -1;
  __amdgpu_buffer_rsrc_t rsa[NA], rsb[NA];
  rsa[0] = __builtin_amdgcn_make_buffer_rsrc((void *)P.a_hi, (short)0, P.a_bytes, 0x00020000);
  rsb[0] = __builtin_amdgcn_make_buffer_rsrc((void *)P.b_hi, (short)0, P.b_bytes, 0x00020000);
  if constexpr (SPLIT) {
    rsa[NA - 1] = __builtin_amdgcn_make_buffer_rsrc((void *)P.a_lo, (short)0, P.a_bytes, 0x00020000);
    rsb[NA - 1] = __builtin_amdgcn_make_buffer_rsrc((void *)P.b_lo, (short)0, P.b_bytes, 0x00020000);
  }
  // FP32: two accumulator sets (even / odd k-steps) per tile; SPLIT: FP64
  constexpr int N32 = SPLIT ? 1 : 2, N64 = SPLIT ? 1 : 0;
  f4 acc[N32][TM][TN];
  d4 acc64[N64 ? TM : 1][N64 ? TN : 1];
#pragma unroll
  for (int t = 0; t < TM; t++)
#pragma unroll
    for (int u = 0; u < TN; u++) {
#pragma unroll
      for (int h = 0; h < N32; h++) acc[h][t][u] = f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (SPLIT) acc64[t][u] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int64_t s0 = P.seg[c], s1 = P.seg[c + 1];
  for (int64_t rbase = s0; rbase < s1; rbase += ROUND) {
    const int nr = (int)min<int64_t>(ROUND, s1 - rbase);
    const int nq = nr >> 2;
    load_quads(P, ql, rbase, nr, lane);
    int steps = 0;
    for (int q = lane; q < nq; q += 64) steps += (ql.Kq[q] + 3) >> 2;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) steps += __shfl_xor(steps, d, 64);
    steps = __builtin_amdgcn_readfirstlane(steps);
    int iq = 0, ip = 0, iP;
    uint32_t va[TM], vb[TN];
    uint32_t noa = QOOB, nob = QOOB;
    int nK = 1 << 20;
    auto lane_offsets = [&](uint32_t oa, uint32_t ob) {
#pragma unroll
      for (int t = 0; t < TM; t++) va[t] = (ra[t] < 0 || oa == QOOB) ? QOOB : oa + 16u * (uint32_t)ra[t];
#pragma unroll
      for (int u = 0; u < TN; u++) vb[u] = (cb[u] < 0 || ob == QOOB) ? QOOB : ob + 16u * (uint32_t)cb[u];
    };
    {
      const int K0 = __builtin_amdgcn_readfirstlane(ql.Kq[0]);
      iP = (K0 + 3) >> 2;
      lane_offsets(ql.oa[kq], ql.ob[kq]);
      if (nq > 1) {
        noa = ql.oa[4 + kq];
        nob = ql.ob[4 + kq];
        nK = ql.Kq[1];
      }
    }
    f4 qa[PF][NA][TM], qb[PF][NA][TN];
    auto issue = [&](f4 (&xa)[NA][TM], f4 (&xb)[NA][TN]) {
      const int sa = ip * m16, sb = ip * n16;
#pragma unroll
      for (int h = 0; h < NA; h++) {
#pragma unroll
        for (int t = 0; t < TM; t++) xa[h][t] = load4(rsa[h], va[t], sa);
#pragma unroll
        for (int u = 0; u < TN; u++) xb[h][u] = load4(rsb[h], vb[u], sb);
      }
      if (++ip == iP) {   // uniform: next quad
        ip = 0;
        iq++;
        const int K = __builtin_amdgcn_readfirstlane(nK);
        iP = (K + 3) >> 2;
        lane_offsets(noa, nob);
        if (iq + 1 < nq) {
          const int t = 4 * (iq + 1) + kq;
          noa = ql.oa[t];
          nob = ql.ob[t];
          nK = ql.Kq[iq + 1];
        } else {
          noa = QOOB;
          nob = QOOB;
          nK = 1 << 20;
        }
      }
    };
    auto mma = [&](const f4 (&xa)[NA][TM], const f4 (&xb)[NA][TN]) {
#pragma unroll
      for (int t = 0; t < TM; t++)
#pragma unroll
        for (int u = 0; u < TN; u++) {
          if constexpr (SPLIT) {
            // one slab (four k-steps): the small terms first, in FP32, then
            // the slab's sum is added to the FP64 accumulator
            f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; e++) {
              z = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[1][t][e], xb[0][u][e], z, 0, 0, 0);
              z = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][t][e], xb[1][u][e], z, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++)
              z = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][t][e], xb[0][u][e], z, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; r++) acc64[t][u][r] += (double)z[r];
          } else {
#pragma unroll
            for (int e = 0; e < 4; e++)
              acc[e % N32][t][u] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][t][e], xb[0][u][e], acc[e % N32][t][u], 0, 0, 0);
          }
        }
    };
#pragma unroll
    for (int d = 0; d < PF; d++) {
      issue(qa[d], qb[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
    int s = 0;
    for (; s + 2 * PF <= steps; s += PF) {
#pragma unroll
      for (int d = 0; d < PF; d++) {
        mma(qa[d], qb[d]);
        issue(qa[d], qb[d]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int d = 0; d < 2 * PF; d++) {
      const int st = s + d;
      if (st < steps) {
        const int slot = d % PF;
        mma(qa[slot], qb[slot]);
        if (st + PF < steps) issue(qa[slot], qb[slot]);
      }
    }
    wave_sync();   // the next round rewrites the parameter LDS
  }

  // epilogue in FP64: C = alpha * acc + beta * C_old, and the block's norm
  const int64_t co = P.c_off[c];
  const double *old = nullptr;
  if (P.beta != 0.0 && P.old_blk) {
    const int32_t ob = P.old_blk[c];
    if (ob >= 0) old = P.old_val + P.old_off[ob];
  }
  double ss = 0.0;
#pragma unroll
  for (int t = 0; t < TM; t++)
#pragma unroll
    for (int u = 0; u < TN; u++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * t + 4 * kq + r, col = 16 * u + l16;
        if (row < m && col < n) {
          double v;
          if constexpr (SPLIT) v = acc64[t][u][r];
          else v = (double)acc[0][t][u][r] + (double)acc[N32 - 1][t][u][r];
          double x = P.alpha * v;
          if (old) x += P.beta * old[row + col * m];
          P.c_val[co + row + (int64_t)col * m] = x;
          ss += x * x;
        }
      }
  if (P.c_norm) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
    if (lane == 0) P.c_norm[c] = sqrt(ss);
  }
}

// BIG: C edges up to 32 (tiles 2x2 compiled in); otherwise up to 16, so the
// register budget (and occupancy) is that of the single-tile case.
template <bool SPLIT, bool BIG>
__global__ __launch_bounds__(64 * WPG) void k_gemm_lowp(LowpP P, int64_t nblk, int64_t chunk) {
  __shared__ QuadLds lds[WPG];
  QuadLds &ql = lds[threadIdx.x >> 6];
  const int64_t b = blockIdx.x;
  const int64_t lb = xcd_logical(b, chunk);
  const int64_t w = lb * WPG + (threadIdx.x >> 6);
  if (w >= nblk) return;   // uniform per wavefront
  const int32_t c = __builtin_amdgcn_readfirstlane(P.c_list ? P.c_list[w] : (int32_t)w);
  if constexpr (!BIG) {
    gemm_block_lowp<SPLIT, 1, 1>(P, c, ql);
  } else {
    const int tm = P.rbs[P.c_row[c]] > 16 ? 2 : 1;
    const int tn = P.cbs[P.c_ci[c]] > 16 ? 2 : 1;
    if (tm == 1 && tn == 1) gemm_block_lowp<SPLIT, 1, 1>(P, c, ql);
    else if (tm == 1) gemm_block_lowp<SPLIT, 1, 2>(P, c, ql);
    else if (tn == 1) gemm_block_lowp<SPLIT, 2, 1>(P, c, ql);
    else gemm_block_lowp<SPLIT, 2, 2>(P, c, ql);
  }
}

// Packed FP32 k-quad slabs of the stored blocks (see the file header):
// stored block (R x C, column-major) viewed as nr rows by K contraction
// indices, slab p = the four k = 4p..4p+3 of every row side by side.
// Offsets are in units of 8 bytes (two floats) so that the stack encoding
// (byte offset = 8 * unit) is shared with the FP64 path.
__global__ __launch_bounds__(64) void k_pack32_sizes(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                    const int32_t *cbs, int k_is_row, int64_t *sizes) {
  const int32_t i = blockIdx.x;
  const int R = rbs[i];
  for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 64) {
    const int C = cbs[ci[p]];
    const int K = k_is_row ? R : C, nr = k_is_row ? C : R;
    sizes[p] = (int64_t)nr * ((K + 3) & ~3) / 2;
  }
}

__global__ __launch_bounds__(256) void k_pack32_blocks(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                       const int32_t *cbs, const int64_t *off, const double *in,
                                                       int k_is_row, const int64_t *poff, float *hi, float *lo) {
  const int32_t i = blockIdx.x;
  const int R = rbs[i];
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const int C = cbs[ci[p]];
    const int K = k_is_row ? R : C, nr = k_is_row ? C : R;
    const int K4 = (K + 3) & ~3;
    const int64_t o = off[p], po = 2 * poff[p];
    for (int e = threadIdx.x; e < nr * K4; e += blockDim.x) {
      const int slab = e / (4 * nr), w = e - slab * 4 * nr;
      const int r = w >> 2, k = 4 * slab + (w & 3);
      double x = 0.0;
      if (k < K) x = k_is_row ? in[o + k + (int64_t)r * R] : in[o + r + (int64_t)k * R];
      const float h = (float)x;
      hi[po + e] = h;
      if (lo) lo[po + e] = (float)(x - (double)h);
    }
  }
}

}  // namespace

void pack32_offsets(Allocator &al, const bsmm_mat_s &x, bool k_is_row, int64_t *d_poff, hipStream_t s) {
  if (x.nnzb == 0) {
    HIPCHECK(hipMemsetAsync(d_poff, 0, sizeof(int64_t), s));
    return;
  }
  DBuf<int64_t> sizes(al, (size_t)x.nnzb);
  hipLaunchKernelGGL(k_pack32_sizes, dim3(x.nbr), dim3(64), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_cbs,
                     k_is_row ? 1 : 0, sizes.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, sizes.p, d_poff, x.nnzb, s);
}

void pack32_values(const bsmm_mat_s &x, bool k_is_row, const int64_t *d_poff, float *hi, float *lo, hipStream_t s) {
  if (x.nbr == 0 || x.nnzb == 0) return;
  hipLaunchKernelGGL(k_pack32_blocks, dim3(x.nbr), dim3(256), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_cbs,
                     x.d_blk_off, x.d_values, k_is_row ? 1 : 0, d_poff, hi, lo);
  HIPCHECK(hipGetLastError());
}

void gemm_launch_lowp(const GemmArgs &g, int64_t nnzb_c, int max_edge, hipStream_t s) {
  if (nnzb_c <= 0) return;
  if (max_edge > 32) fail(BSMM_ERR_UNSUPPORTED, "block size above 32");
  if (!g.quads) fail(BSMM_ERR_UNSUPPORTED, "FP32 / split modes need packed operands below 2 GB and at most 8 k sizes");
  LowpP p;
  p.a_hi = g.a_hi;
  p.a_lo = g.a_lo;
  p.b_hi = g.b_hi;
  p.b_lo = g.b_lo;
  p.a_bytes = (uint32_t)g.a_bytes;
  p.b_bytes = (uint32_t)g.b_bytes;
  p.c_list = g.c_list;
  p.c_row = g.c_row;
  p.c_ci = g.c_ci;
  p.rbs = g.a->rbs;
  p.cbs = g.b->cbs;
  p.c_off = g.c_off;
  p.seg = g.seg_off;
  p.stack = g.stack;
  p.old_blk = g.c_old_blk;
  p.old_off = g.old_off;
  p.old_val = g.old_values;
  p.c_val = g.c_values;
  p.c_norm = g.c_norm;
  p.alpha = g.alpha;
  p.beta = g.beta;
  const int64_t nwg = (nnzb_c + WPG - 1) / WPG;
  const XcdMap xm = xcd_map(nwg);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many C blocks for one launch");
  const bool split = g.mode == BSMM_COMPUTE_SPLIT, big = max_edge > 16;
  if (split && big)
    hipLaunchKernelGGL((k_gemm_lowp<true, true>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else if (split)
    hipLaunchKernelGGL((k_gemm_lowp<true, false>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else if (big)
    hipLaunchKernelGGL((k_gemm_lowp<false, true>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else
    hipLaunchKernelGGL((k_gemm_lowp<false, false>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  HIPCHECK(hipGetLastError());
}

}  // namespace bsmm
