// pack_kernels.hip -- packed operand copies for the quad path of the block
// GEMM (k-pair slabs for FP64), built before every numeric pass.
#include "internal.h"

namespace bsmm {

namespace {

// Packed operand copies for the quad path.  Stored block b (R x C,
// column-major) of X is viewed as nr rows r by K contraction indices k:
//   k_is_row = 1 (op(A) = A^T, op(B) = B):  K = R, nr = C, x(r,k) = in[k + r R]
//   k_is_row = 0 (op(A) = A,   op(B) = B^T): K = C, nr = R, x(r,k) = in[r + k R]
// (for op(A) the rows r are the rows of op(A), for op(B) its columns) and
// stored pair-major: Kp/2 slabs, Kp = K + (K & 1), slab p holding for each
// r the two values x(r, 2p), x(r, 2p+1) (the pad zero).  A lane's 16 bytes
// of slab p are then one 128-bit load giving two k-steps, and the lanes of
// consecutive r read one contiguous run.  Every packed block holds an even
// number of values, so all start 16-byte aligned.
__global__ __launch_bounds__(64) void k_pack_sizes(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                  const int32_t *cbs, int k_is_row, int64_t *sizes) {
  const int32_t i = blockIdx.x;
  const int R = rbs[i];
  for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 64) {
    const int C = cbs[ci[p]];
    const int K = k_is_row ? R : C, nr = k_is_row ? C : R;
    sizes[p] = (int64_t)nr * (K + (K & 1));
  }
}

// One workgroup per block row of A and then of B (one launch for both).  The
// row's blocks are taken 256 at a time: first every thread reads one
// block's sizes and offsets into LDS, then each group of 16 lanes packs
// every 16th block.  A block of at most PACK_STAGE values is read in its
// stored order (contiguous loads), staged in the group's LDS slice, and
// written in packed order (contiguous stores); the packed position of a
// lane (slab, r, k parity) advances by a precomputed stride, without a
// division per value.  Larger blocks are read in packed order directly.
struct PackSide {
  const int64_t *rp;
  const int32_t *ci, *rbs, *cbs;
  const int64_t *off;
  const double *in;
  int k_is_row;
  const int64_t *poff;
  double *out;
  int32_t nbr;
  double *norm;   // optional: Frobenius norm of every stored block
};

constexpr int PACK_NV = 12;                  // values per lane per step
constexpr int PACK_STAGE = 16 * PACK_NV;     // blocks up to this size go through LDS

__device__ inline void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_pack_blocks(PackSide a, PackSide b) {
  __shared__ int64_t m_o[256], m_po[256];
  __shared__ int32_t m_K[256], m_nr[256];
  __shared__ double stage[16][PACK_STAGE];
  const bool first = (int32_t)blockIdx.x < a.nbr;
  const PackSide &X = first ? a : b;
  const int32_t i = first ? (int32_t)blockIdx.x : (int32_t)blockIdx.x - a.nbr;
  const int R = X.rbs[i];
  const int lane = threadIdx.x & 15, grp = threadIdx.x >> 4;
  double *st = stage[grp];
  const int64_t p0 = X.rp[i], p1 = X.rp[i + 1];
  for (int64_t pb = p0; pb < p1; pb += 256) {
    const int nb = (int)min<int64_t>(256, p1 - pb);
    if ((int)threadIdx.x < nb) {
      const int64_t p = pb + threadIdx.x;
      const int C = X.cbs[X.ci[p]];
      m_K[threadIdx.x] = X.k_is_row ? R : C;
      m_nr[threadIdx.x] = X.k_is_row ? C : R;
      m_o[threadIdx.x] = X.off[p];
      m_po[threadIdx.x] = X.poff[p];
    }
    __syncthreads();
    for (int jb = 0; jb < nb; jb += 16) {   // same trip count for every lane
      const int j = jb + grp;
      const bool active = j < nb;
      const int K = active ? m_K[j] : 1, nr = active ? m_nr[j] : 1, two = 2 * nr;
      const int n = active ? nr * (K + (K & 1)) : 0, n_in = nr * K;
      const int64_t o = active ? m_o[j] : 0, po = active ? m_po[j] : 0;
      const bool staged = n_in <= PACK_STAGE;
      // stride of 16 in the packed order: qd slabs and rd more positions
      const int qd = 16 / two, rd = 16 - qd * two;
      int slab = lane / two, w = lane - (lane / two) * two;   // position of e = lane
      // the block norm in the order of the norm kernel: lane sums elements
      // lane, lane + 16, ... of the stored block, then a fixed 16-lane tree
      double ss = 0.0;
      if (active && staged) {
        double x[PACK_NV];
#pragma unroll
        for (int t = 0; t < PACK_NV; t++) x[t] = X.in[o + min(lane + 16 * t, n_in - 1)];
#pragma unroll
        for (int t = 0; t < PACK_NV; t++)
          if (lane + 16 * t < n_in) {
            st[lane + 16 * t] = x[t];
            ss = fma(x[t], x[t], ss);
          }
      } else if (active && X.norm) {
        for (int d = lane; d < n_in; d += 16) {
          const double x = X.in[o + d];
          ss = fma(x, x, ss);
        }
      }
      if (X.norm) {   // uniform: every lane takes part in the tree
#pragma unroll
        for (int dd = 8; dd >= 1; dd >>= 1) ss += __shfl_xor(ss, dd, 16);
        if (active && lane == 0) X.norm[pb + j] = sqrt(ss);
      }
      group_sync();
      if (active && staged) {
        for (int e0 = 0; e0 < n; e0 += 16 * PACK_NV) {
#pragma unroll
          for (int t = 0; t < PACK_NV; t++) {
            const int e = e0 + 16 * t + lane;
            const int k = 2 * slab + (w & 1), r = w >> 1, kc = min(k, K - 1);   // r < nr always
            const double v = st[X.k_is_row ? kc + r * K : r + kc * nr];
            if (e < n) X.out[po + e] = k < K ? v : 0.0;
            slab += qd;
            w += rd;
            if (w >= two) {
              w -= two;
              slab++;
            }
          }
        }
      } else if (active) {
        for (int e0 = 0; e0 < n; e0 += 16 * PACK_NV) {
          double x[PACK_NV];
          int sl[PACK_NV], ww[PACK_NV];
#pragma unroll
          for (int t = 0; t < PACK_NV; t++) {
            sl[t] = slab;
            ww[t] = w;
            const int k = min(2 * slab + (w & 1), K - 1), r = min(w >> 1, nr - 1);
            const int64_t src = X.k_is_row ? o + k + (int64_t)r * R : o + r + (int64_t)k * R;
            x[t] = X.in[src];
            slab += qd;
            w += rd;
            if (w >= two) {
              w -= two;
              slab++;
            }
          }
#pragma unroll
          for (int t = 0; t < PACK_NV; t++) {
            const int e = e0 + 16 * t + lane;
            if (e < n) X.out[po + e] = (2 * sl[t] + (ww[t] & 1) < K) ? x[t] : 0.0;
          }
        }
      }
      group_sync();   // the slice is rewritten by the group's next block
    }
    __syncthreads();
  }
}

// Offsets in unit order: sizes gathered by unit position, and the scanned
// offsets scattered back to the stored blocks.
__global__ __launch_bounds__(256) void k_gather_sizes(int64_t n, const int32_t *blk, const int64_t *in, int64_t *out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = in[blk[t]];
}

__global__ __launch_bounds__(256) void k_scatter_offsets(int64_t n, const int32_t *blk, const int64_t *in,
                                                         int64_t *out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t <= n; t += (int64_t)gridDim.x * blockDim.x)
    out[t < n ? (int64_t)blk[t] : n] = in[t];   // entry n: the total
}

__global__ __launch_bounds__(256) void k_unit_base(int32_t nunits, const int64_t *rp, const int64_t *off,
                                                   int64_t *base) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nunits) base[r] = off[rp[r]];
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

}  // namespace

void pack_offsets_units(Allocator &al, const bsmm_mat_s &x, bool k_is_row, const OpIndex &units, int64_t *d_poff,
                        int64_t *d_base, hipStream_t s) {
  if (x.nnzb == 0) {
    HIPCHECK(hipMemsetAsync(d_poff, 0, sizeof(int64_t), s));
    if (units.nbr > 0) HIPCHECK(hipMemsetAsync(d_base, 0, sizeof(int64_t) * (size_t)units.nbr, s));
    return;
  }
  DBuf<int64_t> sizes(al, (size_t)x.nnzb);
  hipLaunchKernelGGL(k_pack_sizes, dim3(x.nbr), dim3(64), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_cbs,
                     k_is_row ? 1 : 0, sizes.p);
  HIPCHECK(hipGetLastError());
  const int64_t *off = d_poff;
  DBuf<int64_t> usz, uoff;
  if (units.blk) {
    usz = DBuf<int64_t>(al, (size_t)x.nnzb);
    uoff = DBuf<int64_t>(al, (size_t)x.nnzb + 1);
    hipLaunchKernelGGL(k_gather_sizes, dim3(grid_for(x.nnzb)), dim3(256), 0, s, x.nnzb, units.blk, sizes.p, usz.p);
    HIPCHECK(hipGetLastError());
    exclusive_scan_i64(al, usz.p, uoff.p, x.nnzb, s);
    hipLaunchKernelGGL(k_scatter_offsets, dim3(grid_for(x.nnzb + 1)), dim3(256), 0, s, x.nnzb, units.blk, uoff.p,
                       d_poff);
    HIPCHECK(hipGetLastError());
    off = uoff.p;
  } else {
    exclusive_scan_i64(al, sizes.p, d_poff, x.nnzb, s);
  }
  if (units.nbr > 0) {
    hipLaunchKernelGGL(k_unit_base, dim3((unsigned)((units.nbr + 255) / 256)), dim3(256), 0, s, units.nbr,
                       units.row_ptr, off, d_base);
    HIPCHECK(hipGetLastError());
  }
}

void pack_offsets(Allocator &al, const bsmm_mat_s &x, bool k_is_row, int64_t *d_poff, hipStream_t s) {
  if (x.nnzb == 0) {
    HIPCHECK(hipMemsetAsync(d_poff, 0, sizeof(int64_t), s));
    return;
  }
  DBuf<int64_t> sizes(al, (size_t)x.nnzb);
  hipLaunchKernelGGL(k_pack_sizes, dim3(x.nbr), dim3(64), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_cbs,
                     k_is_row ? 1 : 0, sizes.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, sizes.p, d_poff, x.nnzb, s);
}

void pack_values(const bsmm_mat_s &a, bool a_k_is_row, const int64_t *a_poff, double *a_out, const bsmm_mat_s &b,
                 bool b_k_is_row, const int64_t *b_poff, double *b_out, hipStream_t s, double *a_norm,
                 double *b_norm) {
  auto side = [](const bsmm_mat_s &x, bool kr, const int64_t *poff, double *out, double *norm) {
    PackSide v;
    v.rp = x.d_row_ptr;
    v.ci = x.d_col_idx;
    v.rbs = x.d_rbs;
    v.cbs = x.d_cbs;
    v.off = x.d_blk_off;
    v.in = x.d_values;
    v.k_is_row = kr ? 1 : 0;
    v.poff = poff;
    v.out = out;
    v.nbr = (x.nnzb > 0) ? x.nbr : 0;
    v.norm = norm;
    return v;
  };
  const PackSide va = side(a, a_k_is_row, a_poff, a_out, a_norm), vb = side(b, b_k_is_row, b_poff, b_out, b_norm);
  const int64_t grid = (int64_t)va.nbr + vb.nbr;
  if (grid == 0) return;
  hipLaunchKernelGGL(k_pack_blocks, dim3((unsigned)grid), dim3(256), 0, s, va, vb);
  HIPCHECK(hipGetLastError());
}

}  // namespace bsmm
