// gemm_kernels.hip -- batched small-block GEMM on FP64 MFMA (gfx950).
//
// The local multiplication is a batch of small dense block products summed
// into result blocks (arXiv:1705.10218, Section 2).  Here one wavefront owns
// one C block for the whole of its stack segment: the accumulator lives in
// registers, no other wavefront writes that block, and no atomics touch C.
//
// Matrix core: V_MFMA_F64_4X4X4_4B (four independent 4x4x4 FP64 products per
// instruction).  Lane layout on gfx950, checked on the device:
//   A_b[i][k] in lane i + 4b + 16k,  B_b[k][j] in lane j + 4b + 16k,
//   D_b[i][j] in lane j + 4b + 16i.
// A C block of m x n is cut into 4x4 subtiles (MT x NT of them, both even).
// The four MFMA blocks b = 2P + Q take the four quadrants of the subtile
// grid; instruction (u, v) computes subtile (P*MT/2 + u, Q*NT/2 + v) in every
// quadrant at once.  A lane therefore needs MT/2 values of op(A) and NT/2
// values of op(B) per k-step, each reused by NT/2 or MT/2 instructions.
//
// The contraction index is permuted: in k-step kk, lane group kq uses
// k = kq * ks + kk (ks = ceil(K/4)).  Any bijection of k gives the same
// sum; this one makes every lane walk a contiguous run of k, so the
// column-major op(B) operand is read sequentially.  Padded rows, columns and
// k are zero-filled (never loaded), so padding adds no rounding.
#include "internal.h"

namespace bsmm {

namespace {

struct GemmP {
  const int64_t *a_off;
  const double *a_val;
  const int64_t *b_off;
  const double *b_val;
  int ta, tb;
  const int32_t *c_list;
  int64_t first, count;
  const int32_t *c_row, *c_ci;
  const int32_t *rbs, *cbs;   // C block sizes (= op(A) rows, op(B) columns)
  const int64_t *c_off, *seg;
  const int2 *stack;
  const int32_t *old_blk;
  const int64_t *old_off;
  const double *old_val;
  double *c_val;
  double *c_norm;
  double alpha, beta;
};

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmP P) {
  constexpr int HM = MT / 2, HN = NT / 2;
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= P.count) return;   // uniform per wavefront
  const int32_t c = P.c_list ? P.c_list[P.first + w] : (int32_t)(P.first + w);
  const int m = P.rbs[P.c_row[c]];
  const int n = P.cbs[P.c_ci[c]];
  const int L4 = lane & 3;
  const int bq = (lane >> 2) & 3;
  const int kq = lane >> 4;
  const int Pq = bq >> 1, Qq = bq & 1;
  int arow[HM], bcol[HN];
#pragma unroll
  for (int u = 0; u < HM; u++) arow[u] = 4 * (Pq * HM + u) + L4;
#pragma unroll
  for (int v = 0; v < HN; v++) bcol[v] = 4 * (Qq * HN + v) + L4;
  double acc[HM * HN];
#pragma unroll
  for (int t = 0; t < HM * HN; t++) acc[t] = 0.0;

  const int64_t s0 = P.seg[c], s1 = P.seg[c + 1];
  for (int64_t e = s0; e < s1; e++) {
    const int2 ab = P.stack[e];
    const int64_t ao = P.a_off[ab.x];
    const int K = (int)((P.a_off[ab.x + 1] - ao) / m);
    const double *ap = P.a_val + ao;
    const double *bp = P.b_val + P.b_off[ab.y];
    const int ks = (K + 3) >> 2;
    // op(A)[r][k] = ap[r*sar + k*sak], op(B)[k][c] = bp[k*sbk + c*sbc]
    const int sar = P.ta ? K : 1, sak = P.ta ? 1 : m;
    const int sbk = P.tb ? n : 1, sbc = P.tb ? 1 : K;
    for (int kk = 0; kk < ks; kk++) {
      const int k = kq * ks + kk;
      const bool kv = k < K;
      double av[HM], bv[HN];
#pragma unroll
      for (int u = 0; u < HM; u++) av[u] = (kv && arow[u] < m) ? ap[arow[u] * sar + k * sak] : 0.0;
#pragma unroll
      for (int v = 0; v < HN; v++) bv[v] = (kv && bcol[v] < n) ? bp[k * sbk + bcol[v] * sbc] : 0.0;
#pragma unroll
      for (int u = 0; u < HM; u++)
#pragma unroll
        for (int v = 0; v < HN; v++)
          acc[u * HN + v] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[u], bv[v], acc[u * HN + v], 0, 0, 0);
    }
  }

  // epilogue: C = alpha * acc + beta * C_old, column-major, plus the block norm
  const int64_t co = P.c_off[c];
  const double *old = nullptr;
  if (P.beta != 0.0 && P.old_blk) {
    const int32_t ob = P.old_blk[c];
    if (ob >= 0) old = P.old_val + P.old_off[ob];
  }
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < HM; u++) {
    const int row = 4 * (Pq * HM + u) + kq;
#pragma unroll
    for (int v = 0; v < HN; v++) {
      const int col = bcol[v];
      if (row < m && col < n) {
        double x = P.alpha * acc[u * HN + v];
        if (old) x += P.beta * old[row + col * m];
        P.c_val[co + row + (int64_t)col * m] = x;
        ss += x * x;
      }
    }
  }
  if (P.c_norm) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
    if (lane == 0) P.c_norm[c] = sqrt(ss);
  }
}

template <int MT, int NT>
void launch_one(const GemmP &p, hipStream_t s) {
  int64_t blocks = (p.count + 3) / 4;
  hipLaunchKernelGGL((k_gemm_f64<MT, NT>), dim3((unsigned)blocks), dim3(256), 0, s, p);
  HIPCHECK(hipGetLastError());
}

template <int MT>
void launch_nt(const GemmP &p, int nt, hipStream_t s) {
  switch (nt) {
    case 2: launch_one<MT, 2>(p, s); break;
    case 4: launch_one<MT, 4>(p, s); break;
    case 6: launch_one<MT, 6>(p, s); break;
    case 8: launch_one<MT, 8>(p, s); break;
    default: fail(BSMM_ERR_UNSUPPORTED, "block size above 32");
  }
}

}  // namespace

void gemm_launch(const GemmArgs &g, const GemmClass &cls, hipStream_t s) {
  if (cls.count <= 0) return;
  if (cls.count > (int64_t)INT32_MAX * 4) fail(BSMM_ERR_UNSUPPORTED, "too many C blocks in one class");
  GemmP p;
  p.a_off = g.a->blk_off;
  p.a_val = g.a->values;
  p.b_off = g.b->blk_off;
  p.b_val = g.b->values;
  p.ta = g.a->trans ? 1 : 0;
  p.tb = g.b->trans ? 1 : 0;
  p.c_list = g.c_list;
  p.first = cls.first;
  p.count = cls.count;
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
  switch (cls.mt) {
    case 2: launch_nt<2>(p, cls.nt, s); break;
    case 4: launch_nt<4>(p, cls.nt, s); break;
    case 6: launch_nt<6>(p, cls.nt, s); break;
    case 8: launch_nt<8>(p, cls.nt, s); break;
    default: fail(BSMM_ERR_UNSUPPORTED, "block size above 32");
  }
}

}  // namespace bsmm
