// tile_gemm.hip -- block GEMM on tiles of result blocks whose operand blocks
// are staged in LDS and shared by the tile's products.
//
// The local multiplication is a batch of small dense block products summed
// into result blocks (arXiv:1705.10218, Section 2).  Block (i,j) of C needs
// A(i,k) and B(k,j) for every k of its product list, and a neighbouring block
// (i,j') or (i',j) needs most of the same A(i,k) or B(k,j): rows i and i' whose
// atoms are close in space reach nearly the same k.  Here one workgroup owns
// a tile of TI x TJ result blocks (TI rows adjacent in the locality order, TJ
// columns adjacent as well) and walks the union of their product lists in
// ascending k.  At every k the workgroup copies the A(i,k) of its rows and
// the B(k,j) of its columns that some product of the tile uses from the
// stored values into LDS once, and every product of the tile at that k runs
// from LDS: a block fetched from memory serves up to TJ (A) or TI (B)
// products instead of one.  Each of the (TI/2)(TJ/2) wavefronts owns a 2 x 2
// part of the tile.  The copy of step k+1 is in flight (in registers, then
// written to the other of two LDS buffers) while the products of step k run;
// one barrier per step separates them.
//
// The tile path serves result blocks with edges up to 24 (and contraction
// extents up to 24): one V_MFMA_F64_16X16X4F64 tile covers rows and columns
// 0..15, V_MFMA_F64_4X4X4F64 subtiles the edge rows and columns 16..23 of
// blocks that reach them (the edge-subtile layout of the quad path, checked
// element by element on the device).  It is the preferred path for blocks
// with both edges in 17..24 and the path for operands too large for packed
// 32-bit-offset copies; smaller blocks use a fraction of the 16 x 16 tile.  The four k-groups of an MFMA take four
// consecutive k of one block product; K is padded to a multiple of 4 with
// exact zeros.  Stored blocks are read as they are (column-major), so
// transposed operands only change the LDS strides, and 64-bit element
// offsets reach operands of any size: no packed copies.
//
// Each result block keeps a single owner and its accumulators stay in
// registers: no atomics; its products are added in ascending k, identically
// on every run.
#include <cstring>
#include "internal.h"

namespace bsmm {

namespace {

// LDS slot of one operand block: edges up to 24 give at most 576 values;
// a block is copied in 16-byte pairs from the pair boundary at or below its
// first value, so it sits 0 or 1 value into the slot, and the pairs reach
// at most (1 + 576 + 1) / 2 = 289 pairs = 578 values (580: 16-byte slots).
constexpr int TSLOT = 580;
constexpr int NPAIR = 5;    // 64-lane pieces of 16 bytes: 320 >= 289 pairs

// Layouts of one tile shape.
//   descriptor: int32 i[TI], j[TJ], c[TI*TJ] (C block (r, c) at c[r*TJ + c],
//               -1 when not in C), then int64 s0 (first step), int32 ns,
//               padded to 16 bytes;
//   step      : int64 off[TI + TJ] (element offsets of the stored A blocks of
//               rows 0..TI-1, then B blocks of columns 0..TJ-1; -1 unused),
//               int32 K, uint32 mask (bit r*TJ + c: result block (r, c) has
//               a product at this k), padded to 16 bytes.
template <int TI, int TJ>
struct Shape {
  static constexpr int NW = (TI / 2) * (TJ / 2);                // wavefronts
  static constexpr int NS = TI + TJ;                            // LDS slots per buffer
  static constexpr int NB = NW > 1 ? 2 : 1;                     // LDS buffers
  static constexpr int DESC_INTS = TI + TJ + TI * TJ;
  static constexpr int DESC_BYTES = ((DESC_INTS * 4 + 7) / 8 * 8 + 16 + 15) / 16 * 16;
  static constexpr int S0_OFF = (DESC_INTS * 4 + 7) / 8 * 8;   // byte offset of s0
  static constexpr int LPR = NS / 2 + 1;                        // 16-byte lanes per step record
  static constexpr int STEP_BYTES = 16 * LPR;
  static constexpr int RB = 64 / LPR;                           // step records per batch load
  static constexpr int SPW = (NS + NW - 1) / NW;                // blocks a wavefront stages
  static constexpr uint32_t COLBITS = []() {
    uint32_t b = 0;
    for (int r = 0; r < TI; r++) b |= 1u << (r * TJ);
    return b;
  }();
  static __device__ __forceinline__ bool need_a(uint32_t mask, int r) { return (mask >> (r * TJ)) & ((1u << TJ) - 1); }
  static __device__ __forceinline__ bool need_b(uint32_t mask, int c) { return (mask & (COLBITS << c)) != 0; }
};

struct TileP {
  const int4 *tiles;
  const int4 *steps;           // followed by RB readable padding records
  const int32_t *rbs, *cbs;    // C block sizes (rows of op(A), columns of op(B))
  const double *a_val, *b_val; // stored values of A and B
  const double *a_end, *b_end; // one past the last stored value
  int ta, tb;                  // op(A) = A^T, op(B) = B^T
  const int64_t *c_off;
  const int32_t *old_blk;
  const int64_t *old_off;
  const double *old_val;
  double *c_val;
  double *c_norm;
  double alpha, beta;
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <int CTRL, int BANKS = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
  const int2 v = __builtin_bit_cast(int2, x);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(v.x, v.x, CTRL, 0xF, BANKS, false);
  r.y = __builtin_amdgcn_update_dpp(v.y, v.y, CTRL, 0xF, BANKS, false);
  return __builtin_bit_cast(double, r);
}
constexpr int DPP_ROW_SHR4 = 0x114;   // lane l takes lane l - 4 of its row
constexpr int DPP_ROW_ROR4 = 0x124;   // lane l takes lane (l - 4) mod 16 of its row
// row_ror:4 of a double: every lane is written, so no old value is kept
__device__ __forceinline__ double ror4_f64(double x) {
  const int2 v = __builtin_bit_cast(int2, x);
  int2 r;
  r.x = __builtin_amdgcn_mov_dpp(v.x, DPP_ROW_ROR4, 0xF, 0xF, false);
  r.y = __builtin_amdgcn_mov_dpp(v.y, DPP_ROW_ROR4, 0xF, 0xF, false);
  return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ int64_t sread64(const int64_t *p) {
  const int64_t v = *p;
  return ((int64_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int32_t sread32(const int32_t *p) { return __builtin_amdgcn_readfirstlane(*p); }

// RB consecutive step records, 16 bytes per lane.
template <class S>
__device__ __forceinline__ int4 load_batch(const int4 *steps, int64_t first, int lane) {
  return steps[first * S::LPR + min(lane, S::RB * S::LPR - 1)];
}
__device__ __forceinline__ int64_t lane64(int lo, int hi, int l) {
  return ((int64_t)__builtin_amdgcn_readlane(hi, l) << 32) | (uint32_t)__builtin_amdgcn_readlane(lo, l);
}

// A step record: the batch it sits in and its place there; fields are read
// with readlane (a uniform lane index, so no register array is indexed at
// run time).
template <class S>
struct Rec {
  int4 b;
  int l0;   // first lane of the record
  __device__ __forceinline__ void at(const int4 &batch, int t) {
    b = batch;
    l0 = S::LPR * t;
  }
  __device__ __forceinline__ int64_t off(int o) const {   // o uniform, may be a run-time value
    const int l = l0 + (o >> 1);
    return (o & 1) ? lane64(b.z, b.w, l) : lane64(b.x, b.y, l);
  }
  __device__ __forceinline__ int32_t K() const { return __builtin_amdgcn_readlane(b.x, l0 + S::LPR - 1); }
  __device__ __forceinline__ uint32_t mask() const { return (uint32_t)__builtin_amdgcn_readlane(b.y, l0 + S::LPR - 1); }
};

// Where a block is copied from: 16-byte pairs from the pair boundary at or
// below its first value (the block starts `sh` = 0 or 1 values into its
// slot).  A block whose first or last pair would reach outside its array (an
// array that does not start or end on a 16-byte boundary) loads value by
// value inside the array instead.
struct Blk {
  const double *al;   // pair-aligned start
  int np;             // pairs
  int sh;             // values before the block's first in the first pair
  bool edge;          // a pair reaches outside the array
};
__device__ __forceinline__ Blk blk_at(const double *val, const double *end, int64_t off, int sz) {
  Blk b;
  const double *first = val + off;
  b.sh = (int)(((uintptr_t)first >> 3) & 1u);
  b.al = first - b.sh;
  b.np = (b.sh + sz + 1) >> 1;
  b.edge = b.al < val || b.al + 2 * b.np > end;
  return b;
}

template <int TI, int TJ>
__global__ __launch_bounds__((64 * Shape<TI, TJ>::NW)) void k_tile_gemm(TileP P, int64_t ntile, int64_t chunk) {
  using S = Shape<TI, TJ>;
  __shared__ __attribute__((aligned(16))) double slot[S::NB][S::NS][TSLOT];
  const int64_t w = xcd_logical(blockIdx.x, chunk);
  if (w >= ntile) return;   // uniform over the workgroup
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wp = wave / (TJ / 2), wq = wave % (TJ / 2);   // this wavefront's rows 2wp.., columns 2wq..
  const int32_t *td = reinterpret_cast<const int32_t *>(P.tiles + w * (S::DESC_BYTES / 16));
  // lane o < NS: edge of slot o (rows of A row o, or columns of B column o - TI; 0 if absent)
  int edge_v = 0;
  if (lane < S::NS) {
    const int32_t x = td[lane];
    edge_v = x < 0 ? 0 : (lane < TI ? P.rbs[x] : P.cbs[x]);
  }
  auto edge = [&](int o) { return __builtin_amdgcn_readlane(edge_v, o); };
  const int64_t s0 = sread64(reinterpret_cast<const int64_t *>(reinterpret_cast<const char *>(td) + S::S0_OFF));
  const int32_t ns = sread32(reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(td) + S::S0_OFF + 8));
  // this wavefront's two rows (A slots 2wp, 2wp+1) and columns (B slots TI + 2wq ..)
  int mw[2], nw[2];
#pragma unroll
  for (int d = 0; d < 2; d++) {
    mw[d] = edge(2 * wp + d);
    nw[d] = edge(TI + 2 * wq + d);
  }

  const int i16 = lane & 15, kq = lane >> 4, e8 = 16 + (lane & 7);
  d4 acc16[4];
  double acc4[4][5];
#pragma unroll
  for (int x = 0; x < 4; x++) {
    acc16[x] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 5; t++) acc4[x][t] = 0.0;
  }

  // slot o holds A row o (o < TI) or B column o - TI; a wavefront stages
  // slots wave, wave + NW, ...  A step is decoded once into scalars: K,
  // the mask, where this wavefront's staged blocks come from, and the shift
  // of the four blocks its products read.
  struct Step {
    int K;
    uint32_t mask;
    Blk st[S::SPW];    // blocks this wavefront stages (np = 0: not needed)
    int sh[4];         // shifts of A rows 2wp, 2wp+1 and B columns 2wq.., 2wq+1
  };
  auto decode = [&](const int4 &b, int t) {
    Rec<S> R;
    R.at(b, t);
    Step st;
    st.K = R.K();
    st.mask = R.mask();
#pragma unroll
    for (int u = 0; u < S::SPW; u++) {
      const int o = wave + u * S::NW;
      const bool need = o < S::NS && (o < TI ? S::need_a(st.mask, o) : S::need_b(st.mask, o - TI));
      if (need) {
        st.st[u] = o < TI ? blk_at(P.a_val, P.a_end, R.off(o), st.K * edge(o))
                          : blk_at(P.b_val, P.b_end, R.off(o), st.K * edge(o));
      } else {
        st.st[u] = Blk{P.a_val, 0, 0, false};
      }
    }
#pragma unroll
    for (int d = 0; d < 2; d++) {
      st.sh[d] = (int)(((uintptr_t)(P.a_val + R.off(2 * wp + d)) >> 3) & 1u);
      st.sh[2 + d] = (int)(((uintptr_t)(P.b_val + R.off(TI + 2 * wq + d)) >> 3) & 1u);
    }
    return st;
  };
  d2 pre[S::SPW][NPAIR];
  auto fetch = [&](const Step &st) {
#pragma unroll
    for (int u = 0; u < S::SPW; u++) {
      const Blk &q = st.st[u];
      if (q.np > 0) {
        const int o = wave + u * S::NW;
        const double *v0 = o < TI ? P.a_val : P.b_val, *v1 = o < TI ? P.a_end : P.b_end;
        const d2 *src = reinterpret_cast<const d2 *>(q.al);
        if (!q.edge) {
#pragma unroll
          for (int x = 0; x < NPAIR; x++) pre[u][x] = src[min(64 * x + lane, q.np - 1)];
        } else {
#pragma unroll
          for (int x = 0; x < NPAIR; x++) {
            const double *p2 = q.al + 2 * min(64 * x + lane, q.np - 1);
            const double lo = p2 >= v0 ? p2[0] : 0.0;
            const double hi = p2 + 1 < v1 ? p2[1] : 0.0;
            pre[u][x] = d2{lo, hi};
          }
        }
      }
    }
  };
  auto stage = [&](const Step &st, int buf) {
#pragma unroll
    for (int u = 0; u < S::SPW; u++) {
      const Blk &q = st.st[u];
      if (q.np > 0) {
        d2 *dst = reinterpret_cast<d2 *>(&slot[buf][wave + u * S::NW][0]);
#pragma unroll
        for (int x = 0; x < NPAIR; x++) dst[min(64 * x + lane, q.np - 1)] = pre[u][x];
      }
    }
  };

  int4 bcur = int4{0, 0, 0, 0}, bnxt = int4{0, 0, 0, 0};
  Step cur, nxt;
  if (ns > 0) {
    bcur = load_batch<S>(P.steps, s0, lane);
    if (ns > S::RB) bnxt = load_batch<S>(P.steps, s0 + S::RB, lane);
    cur = decode(bcur, 0);
    fetch(cur);
    stage(cur, 0);
    if (S::NW > 1) __syncthreads();
  }
  for (int32_t s = 0; s < ns; s++) {
    const int buf = S::NB > 1 ? (s & 1) : 0;
    const bool more = s + 1 < ns;
    if (more) {   // the next step's blocks go in flight
      const int t = (s + 1) % S::RB;
      if (t == 0) {   // next batch of records; the one after it goes in flight
        bcur = bnxt;
        if (s + 1 + S::RB < ns) bnxt = load_batch<S>(P.steps, s0 + s + 1 + S::RB, lane);
      }
      nxt = decode(bcur, t);
      fetch(nxt);
    }
    const int K = cur.K;
    const uint32_t mask = cur.mask;
    // LDS strides (elements) of op(A) rows / op(B) columns and of k
    int sIa[2], sKa[2], sJb[2], sKb[2];
#pragma unroll
    for (int d = 0; d < 2; d++) {
      sIa[d] = P.ta ? K : 1;
      sKa[d] = P.ta ? 1 : mw[d];
      sJb[d] = P.tb ? 1 : K;
      sKb[d] = P.tb ? nw[d] : 1;
    }
    // this wavefront's products at this k: bit 2r + c for its block (r, c)
    uint32_t mine = 0u;
#pragma unroll
    for (int x = 0; x < 4; x++) mine |= ((mask >> ((2 * wp + (x >> 1)) * TJ + 2 * wq + (x & 1))) & 1u) << x;
    const int nks = (K + 3) >> 2;
    // operand fragments of k-slice ks (four consecutive k, one per k-group);
    // slice ks+1 is read from LDS while the MFMAs of slice ks run
    struct Frag {
      double am[2], ae[2], bm[2], be[2];
    };
    auto read_frag = [&](int ks) {
      Frag f;
      const int k = 4 * ks + kq;
      const bool kv = k < K;
#pragma unroll
      for (int d = 0; d < 2; d++) {
        if ((mine >> (2 * d)) & 3u) {
          const double *sa = &slot[buf][2 * wp + d][cur.sh[d]];
          const double x0 = sa[i16 * sIa[d] + k * sKa[d]];
          const double x1 = sa[e8 * sIa[d] + k * sKa[d]];
          f.am[d] = kv ? x0 : 0.0;
          f.ae[d] = kv ? x1 : 0.0;
        } else {
          f.am[d] = f.ae[d] = 0.0;
        }
        if ((mine >> d) & 5u) {
          const double *sb = &slot[buf][TI + 2 * wq + d][cur.sh[2 + d]];
          const double y0 = sb[k * sKb[d] + i16 * sJb[d]];
          const double y1 = sb[k * sKb[d] + e8 * sJb[d]];
          f.bm[d] = kv ? y0 : 0.0;
          f.be[d] = kv ? y1 : 0.0;
        } else {
          f.bm[d] = f.be[d] = 0.0;
        }
      }
      return f;
    };
    Frag fc = read_frag(0);
    for (int ks = 0; ks < nks; ks++) {
      const Frag fn = read_frag(min(ks + 1, nks - 1));
      double aer[2], ber[2], bes[2];
#pragma unroll
      for (int d = 0; d < 2; d++) {
        aer[d] = dpp_f64<DPP_ROW_ROR4>(fc.ae[d]);
        ber[d] = dpp_f64<DPP_ROW_ROR4>(fc.be[d]);
        bes[d] = dpp_f64<DPP_ROW_SHR4, 0x6>(fc.be[d]);
      }
#pragma unroll
      for (int x = 0; x < 4; x++) {
        const int r = x >> 1, c = x & 1;
        if ((mine >> x) & 1u) {
          // edge subtiles only where the block reaches past 16 rows / columns
          acc16[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(fc.am[r], fc.bm[c], acc16[x], 0, 0, 0);
          if (nw[c] > 16) {
            acc4[x][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(fc.am[r], fc.be[c], acc4[x][0], 0, 0, 0);
            acc4[x][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(fc.am[r], ber[c], acc4[x][1], 0, 0, 0);
          }
          if (mw[r] > 16) {
            acc4[x][2] = __builtin_amdgcn_mfma_f64_4x4x4f64(fc.ae[r], fc.bm[c], acc4[x][2], 0, 0, 0);
            acc4[x][3] = __builtin_amdgcn_mfma_f64_4x4x4f64(aer[r], fc.bm[c], acc4[x][3], 0, 0, 0);
          }
          if (mw[r] > 16 && nw[c] > 16)
            acc4[x][4] = __builtin_amdgcn_mfma_f64_4x4x4f64(fc.ae[r], bes[c], acc4[x][4], 0, 0, 0);
        }
      }
      fc = fn;
    }
    if (more) {
      // the other buffer was last read before the previous barrier (one
      // wavefront: the same buffer, after this step's reads, in LDS order)
      stage(nxt, S::NB > 1 ? (buf ^ 1) : 0);
      cur = nxt;
    }
    if (S::NW > 1) __syncthreads();
  }

  // epilogue: C = alpha * acc + beta * C_old for every result block of this
  // wavefront's part, and its Frobenius norm for the post-filter
  const int i4 = lane >> 4, j4 = lane & 3, b4 = (lane >> 2) & 3, lo = b4 & 1;
#pragma unroll
  for (int x = 0; x < 4; x++) {
    const int r = x >> 1, c = x & 1;
    const int32_t cb = sread32(td + TI + TJ + (2 * wp + r) * TJ + 2 * wq + c);
    if (cb < 0) continue;
    const int m = mw[r], n = nw[c];
    const int64_t co = sread64(P.c_off + cb);
    const double *old = nullptr;
    if (P.beta != 0.0 && P.old_blk) {
      const int32_t ob = sread32(P.old_blk + cb);
      if (ob >= 0) old = P.old_val + sread64(P.old_off + ob);
    }
    double ss = 0.0;
    auto put = [&](int row, int col, double v) {
      if (row < m && col < n) {
        double y = P.alpha * v;
        if (old) y += P.beta * old[row + (int64_t)col * m];
        P.c_val[co + row + (int64_t)col * m] = y;
        ss += y * y;
      }
    };
#pragma unroll
    for (int t = 0; t < 4; t++) put(4 * t + kq, i16, acc16[x][t]);
    put(4 * b4 + i4, 16 + 4 * lo + j4, acc4[x][0]);
    put(4 * b4 + i4, 16 + 4 * (lo ^ 1) + j4, acc4[x][1]);
    put(16 + 4 * lo + i4, 4 * b4 + j4, acc4[x][2]);
    put(16 + 4 * (lo ^ 1) + i4, 4 * b4 + j4, acc4[x][3]);
    put(16 + 4 * lo + i4, 16 + 4 * (b4 >> 1) + j4, acc4[x][4]);
    if (P.c_norm) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
      if (lane == 0) P.c_norm[cb] = sqrt(ss);
    }
  }
}

// ------------------------------------------------------------ tile plan
__device__ inline int32_t bsearch_pos(const int32_t *ci, int64_t lo, int64_t hi, int32_t j) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    const int32_t v = ci[mid];
    if (v == j) return (int32_t)mid;
    if (v < j) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// flag = 1 if some block p of an array does not start at element p * area
// (stored blocks all of one area, in storage order: it starts there).
__global__ __launch_bounds__(256) void k_off_irregular(const int64_t *off, int64_t n, int64_t area, int32_t *flag) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    if (off[p] != area * p) *flag = 1;
}

// Row groups of the tile plan: group g holds the TI rows x = TI g .. of the
// order ord (the rows of its tiles).  k_group_len: the number of op(A)
// entries of each group's rows, and the largest such number.
template <int TI>
__global__ __launch_bounds__(256) void k_group_len(const int32_t *ord, int32_t nbr, int32_t ngroup, const int64_t *arp,
                                                   int64_t *glen, unsigned long long *gmax) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroup) return;
  int64_t n = 0;
  for (int r = 0; r < TI; r++) {
    const int32_t x = TI * g + r;
    if (x >= nbr) break;
    const int32_t row = ord ? ord[x] : x;
    n += arp[row + 1] - arp[row];
  }
  glen[g] = n;
  atomicMax(gmax, (unsigned long long)n);
}

// The k of a row group's op(A) entries in compact form: ukey[gbase[g] + u]
// is the u-th smallest of them, ucount[g] their number, and upos[a] = u for
// every stored A block a of the group's rows.  The step builder then keeps
// its bitmaps over a group's u (about a row's length) instead of over every
// k.  One workgroup per group: a bitmap over k in LDS and its prefix
// popcounts.
template <int TI>
__global__ __launch_bounds__(256) void k_group_union(const int32_t *ord, int32_t nbr, const int64_t *arp,
                                                     const int32_t *aci, const int32_t *ablk, int32_t nbk,
                                                     const int64_t *gbase, int32_t *ukey, int32_t *upos,
                                                     int32_t *ucount) {
  extern __shared__ uint32_t sm[];
  __shared__ int32_t wsum[4];
  const int32_t g = blockIdx.x;
  const int32_t W = (nbk + 31) >> 5;
  uint32_t *bm = sm;
  int32_t *pre = reinterpret_cast<int32_t *>(sm + W);
  for (int32_t t = threadIdx.x; t < W; t += blockDim.x) bm[t] = 0u;
  __syncthreads();
  for (int r = 0; r < TI; r++) {
    const int32_t x = TI * g + r;
    if (x >= nbr) break;
    const int32_t row = ord ? ord[x] : x;
    for (int64_t p = arp[row] + threadIdx.x; p < arp[row + 1]; p += blockDim.x) {
      const int32_t k = aci[p];
      atomicOr(&bm[k >> 5], 1u << (k & 31));
    }
  }
  __syncthreads();
  // exclusive prefix of the words' popcounts (contiguous words per thread)
  const int32_t per = (W + blockDim.x - 1) / blockDim.x;
  const int32_t w0 = min(W, (int32_t)threadIdx.x * per), w1 = min(W, w0 + per);
  int32_t loc = 0;
  for (int32_t t = w0; t < w1; t++) loc += __popc(bm[t]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t run = inc - loc, total = 0;
  for (int x = 0; x < (int)(blockDim.x >> 6); x++) {
    if (x < wv) run += wsum[x];
    total += wsum[x];
  }
  const int64_t base = gbase[g];
  for (int32_t t = w0; t < w1; t++) {
    pre[t] = run;
    uint32_t word = bm[t];
    while (word) {
      ukey[base + run] = 32 * t + __builtin_ctz(word);
      word &= word - 1;
      run++;
    }
  }
  if (threadIdx.x == 0) ucount[g] = total;
  __syncthreads();
  for (int r = 0; r < TI; r++) {
    const int32_t x = TI * g + r;
    if (x >= nbr) break;
    const int32_t row = ord ? ord[x] : x;
    for (int64_t p = arp[row] + threadIdx.x; p < arp[row + 1]; p += blockDim.x) {
      const int32_t k = aci[p];
      upos[ablk ? ablk[p] : (int32_t)p] = pre[k >> 5] + __popc(bm[k >> 5] & ((1u << (k & 31)) - 1u));
    }
  }
}

// Tiles of row block q: RG consecutive row groups of TI rows of the order
// ord (rows ord[TI (RG q + g) + r]).  A bitmap per row group over column
// groups (group of column j = crank[j] / TJ) in LDS; the tiles of the block
// are the (row group, column group) pairs with a result block, ordered by
// column group, then row group.  One row group per block (RG = 1): the
// tiles that run at the same time on an XCD share their rows' A blocks; 16
// row groups per block, so that they would share B columns as well, halved
// the L2 hit rate of the 23x23 GEMM on a 20,000-atom panel (34 % -> 21 %)
// and slowed it by 9 %.  count mode writes the block's tile count; fill mode
// writes its descriptors from tile_off[q].
constexpr int RG = 1;
template <int TI, int TJ>
__global__ __launch_bounds__(256) void k_tile_groups(const int32_t *ord, int32_t nbr, const int64_t *c_rp,
                                                     const int32_t *c_ci, const int32_t *crank,
                                                     const int32_t *cinv, int32_t nbc, int64_t *count,
                                                     const int64_t *tile_off, int4 *tiles) {
  using S = Shape<TI, TJ>;
  extern __shared__ uint32_t bm[];   // RG bitmaps of W words
  __shared__ int32_t wsum[4];
  const int32_t q = blockIdx.x;
  const int32_t ncg = (nbc + TJ - 1) / TJ;
  const int32_t W = (ncg + 31) >> 5;
  for (int32_t t = threadIdx.x; t < RG * W; t += blockDim.x) bm[t] = 0u;
  __syncthreads();
  for (int g = 0; g < RG; g++) {
    for (int r = 0; r < TI; r++) {
      const int32_t x = TI * (RG * q + g) + r;
      if (x >= nbr) break;
      const int32_t row = ord ? ord[x] : x;
      for (int64_t e = c_rp[row] + threadIdx.x; e < c_rp[row + 1]; e += blockDim.x) {
        const int32_t j = c_ci[e];
        const int32_t p = (crank ? crank[j] : j) / TJ;
        atomicOr(&bm[g * W + (p >> 5)], 1u << (p & 31));
      }
    }
  }
  __syncthreads();
  // per-thread contiguous words, prefix of their tile counts
  const int32_t per = (W + blockDim.x - 1) / blockDim.x;
  const int32_t w0 = min(W, (int32_t)threadIdx.x * per), w1 = min(W, w0 + per);
  int32_t loc = 0;
  for (int32_t t = w0; t < w1; t++)
    for (int g = 0; g < RG; g++) loc += __popc(bm[g * W + t]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t run = inc - loc, total = 0;
  for (int x = 0; x < (int)(blockDim.x >> 6); x++) {
    if (x < wv) run += wsum[x];
    total += wsum[x];
  }
  if (count) {
    if (threadIdx.x == 0) count[q] = total;
    return;
  }
  const int64_t base = tile_off[q];
  for (int32_t t = w0; t < w1; t++) {
    uint32_t any = 0u;
    for (int g = 0; g < RG; g++) any |= bm[g * W + t];
    while (any) {
      const int b = __builtin_ctz(any);
      any &= any - 1;
      const int32_t p = 32 * t + b;
      int32_t cols[TJ];
#pragma unroll
      for (int c = 0; c < TJ; c++) {
        const int32_t x = TJ * p + c;
        cols[c] = x < nbc ? (cinv ? cinv[x] : x) : -1;
      }
      for (int g = 0; g < RG; g++) {
        if (!((bm[g * W + t] >> b) & 1u)) continue;
        int32_t *d = reinterpret_cast<int32_t *>(tiles + (base + run) * (S::DESC_BYTES / 16));
        d[(S::S0_OFF + 12) / 4] = RG * q + g;   // the tile's row group (after s0 and the step count)
#pragma unroll
        for (int c = 0; c < TJ; c++) d[TI + c] = cols[c];
#pragma unroll
        for (int r = 0; r < TI; r++) {
          const int32_t x = TI * (RG * q + g) + r;
          const int32_t i = x < nbr ? (ord ? ord[x] : x) : -1;
          d[r] = i;
#pragma unroll
          for (int c = 0; c < TJ; c++) {
            const int32_t j = cols[c];
            d[TI + TJ + r * TJ + c] = (i >= 0 && j >= 0) ? bsearch_pos(c_ci, c_rp[i], c_rp[i + 1], j) : -1;
          }
        }
        run++;
      }
    }
  }
}

// Union of the k of a tile's product lists: per result block x of the tile a
// bitmap over the compact k of its row group (k_group_union) in LDS, their
// union, and the union's prefix popcounts.  One wavefront per tile.  count
// mode: the number of steps into count[t].  fill mode: the step records from
// the tile's s0 -- for step s (the s-th k of the union): the element offsets
// of the A and B blocks the tile's products use at that k, K and the mask of
// result blocks with a product at this k.  a_area / b_area: the one block area
// of A / B when block p starts at p times it (checked when the plan is built),
// else 0 and the offsets are read from a_off / b_off.
template <int TI, int TJ>
__global__ __launch_bounds__(64) void k_tile_steps(int4 *tiles, int64_t ntile, const int64_t *seg,
                                                   const int2 *stack, const int32_t *upos, const int32_t *ukey,
                                                   const int32_t *ucount, const int64_t *gbase,
                                                   const int32_t *ksz, const int64_t *a_off, const int64_t *b_off,
                                                   int64_t a_area, int64_t b_area, int64_t *count,
                                                   const int64_t *step_off, int4 *steps, int64_t chunk) {
  using S = Shape<TI, TJ>;
  constexpr int NX = TI * TJ;
  extern __shared__ uint32_t sm[];
  const int64_t t = xcd_logical(blockIdx.x, chunk);
  if (t >= ntile) return;
  const int lane = threadIdx.x;
  int32_t *td = reinterpret_cast<int32_t *>(tiles + t * (S::DESC_BYTES / 16));
  const int32_t grp = td[(S::S0_OFF + 12) / 4];   // the tile's row group
  const int32_t W = (ucount[grp] + 31) >> 5;       // words over the group's compact k
  const int32_t *gkey = ukey + gbase[grp];
  const bool fill = count == nullptr;
  uint32_t *bmx = sm;                 // NX x W
  uint32_t *un = sm + NX * W;         // W
  int32_t *pre = reinterpret_cast<int32_t *>(sm + (NX + 1) * W);   // W
  for (int32_t u = lane; u < NX * W; u += 64) bmx[u] = 0u;
  // the tile's product lists as one index range: entry i (0 <= i < tot) is
  // stack entry sb[x] + i - lo[x] of result block x, lo[x] <= i < lo[x + 1];
  // each lane takes CH entries at a time, so their loads are in flight together
  constexpr int CH = 8;
  int64_t sb[NX];
  int32_t lo[NX + 1];
  lo[0] = 0;
#pragma unroll
  for (int x = 0; x < NX; x++) {
    const int32_t cb = td[TI + TJ + x];
    int64_t b0 = 0, b1 = 0;
    if (cb >= 0) {
      b0 = seg[cb];
      b1 = seg[cb + 1];
    }
    sb[x] = b0;
    lo[x + 1] = lo[x] + (int32_t)(b1 - b0);
  }
  const int32_t tot = lo[NX];
  auto locate = [&](int32_t i, int &x) {   // the last x with lo[x] <= i: the one holding i
    int64_t e = sb[0] + i;
    x = 0;
#pragma unroll
    for (int y = 1; y < NX; y++)
      if (i >= lo[y]) {
        x = y;
        e = sb[y] + (i - lo[y]);
      }
    return e;
  };
  // entries i0, i0 + 64, ...: stored A and B block of each, its result block
  // (-1 past the end) and its compact k
  auto gather = [&](int32_t i0, int2 (&pr)[CH], int (&xs)[CH], int32_t (&kk)[CH]) {
#pragma unroll
    for (int u = 0; u < CH; u++) {
      const int32_t i = i0 + 64 * u;
      xs[u] = -1;
      if (i < tot) pr[u] = stack[locate(i, xs[u])];
    }
#pragma unroll
    for (int u = 0; u < CH; u++)
      if (xs[u] >= 0) kk[u] = upos[pr[u].x];
  };
  __syncthreads();
  // the first chunk stays in registers for the pass that writes the steps
  int2 pr0[CH];
  int xs0[CH];
  int32_t kk0[CH];
  gather(lane, pr0, xs0, kk0);
#pragma unroll
  for (int u = 0; u < CH; u++)
    if (xs0[u] >= 0) atomicOr(&bmx[xs0[u] * W + (kk0[u] >> 5)], 1u << (kk0[u] & 31));
  for (int32_t i0 = lane + CH * 64; i0 < tot; i0 += CH * 64) {
    int2 pr[CH];
    int xs[CH];
    int32_t kk[CH];
    gather(i0, pr, xs, kk);
#pragma unroll
    for (int u = 0; u < CH; u++)
      if (xs[u] >= 0) atomicOr(&bmx[xs[u] * W + (kk[u] >> 5)], 1u << (kk[u] & 31));
  }
  __syncthreads();
  const int32_t per = (W + 63) / 64;
  const int32_t w0 = min(W, lane * per), w1 = min(W, w0 + per);
  int32_t loc = 0;
  for (int32_t u = w0; u < w1; u++) {
    uint32_t v = 0u;
    for (int x = 0; x < NX; x++) v |= bmx[x * W + u];
    un[u] = v;
    loc += __popc(v);
  }
  int32_t inc = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  const int32_t total = __shfl(inc, 63, 64);
  if (!fill) {
    if (lane == 0) count[t] = total;
    return;
  }
  int32_t run = inc - loc;
  for (int32_t u = w0; u < w1; u++) {
    pre[u] = run;
    run += __popc(un[u]);
  }
  __syncthreads();
  const int64_t base = step_off[t];
  if (lane == 0) {
    *reinterpret_cast<int64_t *>(reinterpret_cast<char *>(td) + S::S0_OFF) = base;
    *reinterpret_cast<int32_t *>(reinterpret_cast<char *>(td) + S::S0_OFF + 8) = total;
  }
  // per step: K, the mask, -1 for the A rows / B columns the step does not use
  for (int32_t u = w0; u < w1; u++) {
    uint32_t word = un[u];
    int32_t s = pre[u];
    while (word) {
      const int b = __builtin_ctz(word);
      word &= word - 1;
      const int32_t k = 32 * u + b;
      uint32_t mask = 0u;
      for (int x = 0; x < NX; x++) mask |= ((bmx[x * W + u] >> b) & 1u) << x;
      int64_t *r = reinterpret_cast<int64_t *>(steps + (base + s) * S::LPR);
      int32_t *tail = reinterpret_cast<int32_t *>(r + S::NS);
      tail[0] = ksz[gkey[k]];
      tail[1] = (int32_t)mask;
      tail[2] = tail[3] = 0;
#pragma unroll
      for (int o = 0; o < S::NS; o++)
        if (!(o < TI ? S::need_a(mask, o) : S::need_b(mask, o - TI))) r[o] = -1;
      s++;
    }
  }
  // the blocks the steps use (result blocks of one row or column write the
  // same offset)
  auto place = [&](const int2 (&pr)[CH], const int (&xs)[CH], const int32_t (&kk)[CH]) {
#pragma unroll
    for (int u = 0; u < CH; u++) {
      if (xs[u] < 0) continue;
      const int r = xs[u] / TJ, c = xs[u] % TJ;
      const int32_t k = kk[u], w = k >> 5;
      const int32_t s = pre[w] + __popc(un[w] & ((1u << (k & 31)) - 1u));
      int64_t *rr = reinterpret_cast<int64_t *>(steps + (base + s) * S::LPR);
      rr[r] = a_area ? a_area * pr[u].x : a_off[pr[u].x];
      rr[TI + c] = b_area ? b_area * pr[u].y : b_off[pr[u].y];
    }
  };
  place(pr0, xs0, kk0);
  for (int32_t i0 = lane + CH * 64; i0 < tot; i0 += CH * 64) {
    int2 pr[CH];
    int xs[CH];
    int32_t kk[CH];
    gather(i0, pr, xs, kk);
    place(pr, xs, kk);
  }
}

// Products of every tile (the sum of its result blocks' stack segments):
// a bound on its steps, the union of their k.
template <int TI, int TJ>
__global__ __launch_bounds__(256) void k_tile_bound(const int4 *tiles, int64_t ntile, const int64_t *seg,
                                                    int64_t *out) {
  using S = Shape<TI, TJ>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntile) return;
  const int32_t *td = reinterpret_cast<const int32_t *>(tiles + t * (S::DESC_BYTES / 16));
  int64_t n = 0;
  for (int x = 0; x < TI * TJ; x++) {
    const int32_t cb = td[TI + TJ + x];
    if (cb >= 0) n += seg[cb + 1] - seg[cb];
  }
  out[t] = n;
}

template <int TI, int TJ>
void build_plan_t(Allocator &al, const int32_t *ord, const int32_t *crank, const int32_t *cinv, int32_t nbr,
                  int32_t nbc, const int64_t *c_rp, const int32_t *c_ci, const int64_t *seg, const int2 *stack,
                  const OpRows &ar, int32_t nbk, const int32_t *ksz, const int64_t *a_off, const int64_t *b_off,
                  OffsetAreas ob, int64_t *pinned, TilePlan &tp, hipStream_t s) {
  using S = Shape<TI, TJ>;
  const int32_t ngroup = (nbr + TI * RG - 1) / (TI * RG);   // row blocks
  tp.ntile = tp.nsteps = 0;
  if (ngroup == 0) return;
  // tiles
  const int32_t ncg = (nbc + TJ - 1) / TJ;
  const size_t lds = sizeof(uint32_t) * RG * (size_t)std::max((ncg + 31) >> 5, 1);
  if (lds > 65536)
    HIPCHECK(hipFuncSetAttribute((const void *)k_tile_groups<TI, TJ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
  DBuf<int64_t> cnt(al, ngroup), off(al, (size_t)ngroup + 1);
  hipLaunchKernelGGL((k_tile_groups<TI, TJ>), dim3(ngroup), dim3(256), lds, s, ord, nbr, c_rp, c_ci, crank, cinv,
                     nbc, cnt.p, (const int64_t *)nullptr, (int4 *)nullptr);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, cnt.p, off.p, ngroup, s);
  // the compact k of every row group (its rows' op(A) entries, at most)
  DBuf<int64_t> glen(al, ngroup), gbase(al, (size_t)ngroup + 1);
  DBuf<unsigned long long> gmax(al, 1);
  HIPCHECK(hipMemsetAsync(gmax.p, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL((k_group_len<TI>), dim3((unsigned)((ngroup + 255) / 256)), dim3(256), 0, s, ord, nbr, ngroup,
                     ar.rp, glen.p, gmax.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, glen.p, gbase.p, ngroup, s);
  const size_t lds_u = sizeof(uint32_t) * 2 * (size_t)std::max((nbk + 31) >> 5, 1);
  if (lds_u > 65536)
    HIPCHECK(hipFuncSetAttribute((const void *)k_group_union<TI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_u));
  DBuf<int32_t> ukey(al, (size_t)std::max<int64_t>(ar.nnzb, 1)), upos(al, (size_t)std::max<int64_t>(ar.nnzb, 1)),
      ucount(al, ngroup);
  hipLaunchKernelGGL((k_group_union<TI>), dim3(ngroup), dim3(256), lds_u, s, ord, nbr, ar.rp, ar.ci, ar.blk, nbk,
                     gbase.p, ukey.p, upos.p, ucount.p);
  HIPCHECK(hipGetLastError());
  // A and B blocks of one area each: do their offsets follow from it?
  DBuf<int32_t> irregular(al, 2);
  HIPCHECK(hipMemsetAsync(irregular.p, 0, 2 * sizeof(int32_t), s));
  const int64_t areas[2] = {ob.a_area, ob.b_area}, nblk[2] = {ob.a_n, ob.b_n};
  const int64_t *offs[2] = {a_off, b_off};
  for (int x = 0; x < 2; x++)
    if (areas[x] > 0 && nblk[x] > 0) {
      hipLaunchKernelGGL(k_off_irregular, dim3((unsigned)std::min<int64_t>((nblk[x] + 255) / 256, 8192)), dim3(256), 0,
                         s, offs[x], nblk[x], areas[x], irregular.p + x);
      HIPCHECK(hipGetLastError());
    }
  HIPCHECK(hipMemcpyAsync(pinned, off.p + ngroup, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(pinned + 1, gmax.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(pinned + 2, irregular.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  int32_t irr[2];
  std::memcpy(irr, pinned + 2, sizeof(irr));
  const int64_t a_area = (ob.a_area > 0 && !irr[0]) ? ob.a_area : 0;
  const int64_t b_area = (ob.b_area > 0 && !irr[1]) ? ob.b_area : 0;
  const int64_t nt = pinned[0];
  const int64_t wgroup = std::min<int64_t>((nbk + 31) >> 5, (pinned[1] + 31) >> 5);   // words of the widest group
  tp.ntile = nt;
  tp.tiles = DBuf<int4>(al, (size_t)std::max<int64_t>(nt, 1) * (S::DESC_BYTES / 16));
  if (nt <= 0) return;
  hipLaunchKernelGGL((k_tile_groups<TI, TJ>), dim3(ngroup), dim3(256), lds, s, ord, nbr, c_rp, c_ci, crank, cinv,
                     nbc, (int64_t *)nullptr, (const int64_t *)off.p, tp.tiles.p);
  HIPCHECK(hipGetLastError());
  // step records
  const size_t lds2 = sizeof(uint32_t) * (TI * TJ + 2) * (size_t)std::max<int64_t>(wgroup, 1);
  if (lds2 > 65536)
    HIPCHECK(hipFuncSetAttribute((const void *)k_tile_steps<TI, TJ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds2));
  const XcdMap xm = xcd_map(nt);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many result tiles for one launch");
  // Where the records go: a tile has at most as many steps as products, so
  // laid out by that bound the records are written in one pass.  When the
  // bound takes more than 64 GiB or a quarter of what the budget leaves,
  // the steps are counted first and laid out exactly.
  DBuf<int64_t> tcnt(al, (size_t)nt), toff(al, (size_t)nt + 1);
  hipLaunchKernelGGL((k_tile_bound<TI, TJ>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, tp.tiles.p, nt, seg,
                     tcnt.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, tcnt.p, toff.p, nt, s);
  HIPCHECK(hipMemcpyAsync(pinned, toff.p + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const double bound_bytes = (double)pinned[0] * S::LPR * 16.0;
  if (bound_bytes > 64.0 * (double)(1ull << 30) || bound_bytes > 0.25 * (double)al.room()) {
    hipLaunchKernelGGL((k_tile_steps<TI, TJ>), dim3((unsigned)grid), dim3(64), lds2, s, tp.tiles.p, nt, seg, stack,
                       upos.p, ukey.p, ucount.p, gbase.p, ksz, a_off, b_off, a_area, b_area, tcnt.p,
                       (const int64_t *)nullptr, (int4 *)nullptr, xm.chunk);
    HIPCHECK(hipGetLastError());
    exclusive_scan_i64(al, tcnt.p, toff.p, nt, s);
    HIPCHECK(hipMemcpyAsync(pinned, toff.p + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  tp.nsteps = pinned[0];   // records laid out (steps, or the products bound)
  // RB records of padding: a batch load at a tile's last steps reads past them
  tp.steps = DBuf<int4>(al, ((size_t)std::max<int64_t>(tp.nsteps, 0) + S::RB) * S::LPR);
  hipLaunchKernelGGL((k_tile_steps<TI, TJ>), dim3((unsigned)grid), dim3(64), lds2, s, tp.tiles.p, nt, seg, stack,
                     upos.p, ukey.p, ucount.p, gbase.p, ksz, a_off, b_off, a_area, b_area, (int64_t *)nullptr,
                     (const int64_t *)toff.p, tp.steps.p, xm.chunk);
  HIPCHECK(hipGetLastError());
}

template <int TI, int TJ>
void launch_t(const TilePlan &tp, const TileP &p, int64_t max_chunk, hipStream_t s) {
  using S = Shape<TI, TJ>;
  const XcdMap xm = xcd_map(tp.ntile, max_chunk);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many result tiles for one launch");
  hipLaunchKernelGGL((k_tile_gemm<TI, TJ>), dim3((unsigned)grid), dim3(64 * S::NW), 0, s, p, tp.ntile, xm.chunk);
  HIPCHECK(hipGetLastError());
}


// ------------------------------------------------ uniform block size
// Every block of op(A), op(B) and C is S x S (S fixed at compile time, 17..24:
// the uniform-size case, e.g. one basis size per atom).  One wavefront owns a
// 2 x 2 tile as above, but with every extent known the step needs no size
// decoding, the LDS fragment offsets are immediates, and each of the 24
// MFMAs of a k-slice is issued without a branch when all four result blocks
// have a product at the step's k (with per-product branches otherwise).
// A block is copied as NP = ceil(S^2 / 2) 16-byte pieces read from its
// first value on (8-byte aligned loads); when S^2 is odd the last piece is
// read one value earlier, so no load leaves the block, and its upper value
// is moved down.  Slots then start on a 16-byte boundary (no shift).
template <int S>
struct Uni {
  static constexpr int NV = S * S;
  static constexpr int NP = (NV + 1) / 2;      // 16-byte pieces of a block
  static constexpr int NL = (NP + 63) / 64;    // pieces per lane
  static constexpr int NKS = (S + 3) / 4;      // k-slices
  static constexpr int KT = S - 4 * (NKS - 1); // k-groups of the last slice that hold a k
  static constexpr int SLOT = 2 * NP;          // doubles of an LDS slot
};

typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// One tile w of the uniform-size kernel (slot: the wavefront's LDS).
template <int S, bool TA, bool TB>
__device__ __forceinline__ void tile_uni(const TileP &P, int64_t w, double (&slot)[4][Uni<S>::SLOT]) {
  using SH = Shape<2, 2>;
  using U = Uni<S>;
  static_assert(S >= 17 && S <= 24, "the edge subtiles cover rows and columns 16..23");
  const int lane = threadIdx.x;
  const int32_t *td = reinterpret_cast<const int32_t *>(P.tiles + w * (SH::DESC_BYTES / 16));
  const int64_t s0 = sread64(reinterpret_cast<const int64_t *>(reinterpret_cast<const char *>(td) + SH::S0_OFF));
  const int32_t ns = sread32(reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(td) + SH::S0_OFF + 8));

  // element (i, k) of op(A) and (k, j) of op(B) within a slot
  auto ao = [](int i, int k) { return TA ? k + i * S : i + k * S; };
  auto bo = [](int k, int j) { return TB ? j + k * S : k + j * S; };
  const int i16 = lane & 15, kq = lane >> 4;
  const int e8 = min(16 + (lane & 7), S - 1);   // rows / columns >= S are computed and discarded
  const int am0 = ao(i16, kq), ae0 = ao(e8, kq), bm0 = bo(kq, i16), be0 = bo(kq, e8);
  // the last slice: k-groups past S read k = S - 1 and take zeros
  const int kl = min(4 * (U::NKS - 1) + kq, S - 1);
  const int aml = ao(i16, kl), ael = ao(e8, kl), bml = bo(kl, i16), bel = bo(kl, e8);
  const bool kval = kq < U::KT;

  d4 acc16[4];
  double acc4[4][5];
#pragma unroll
  for (int x = 0; x < 4; x++) {
    acc16[x] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 5; t++) acc4[x][t] = 0.0;
  }

  d2 pre[4][U::NL];
  auto need = [](uint32_t mask, int o) { return o < 2 ? SH::need_a(mask, o) : SH::need_b(mask, o - 2); };
  auto fetch = [&](const Rec<SH> &R, uint32_t mask) {
#pragma unroll
    for (int o = 0; o < 4; o++) {
      if (need(mask, o)) {
        const double *first = (o < 2 ? P.a_val : P.b_val) + R.off(o);
#pragma unroll
        for (int x = 0; x < U::NL; x++) {
          const int p = 64 * x + lane;
          if (x < U::NL - 1 || p < U::NP) {
            // only the last piece of a block of odd size is read one value early
            const int e = (x == U::NL - 1 && (U::NV & 1) && p == U::NP - 1) ? U::NV - 2 : 2 * p;
            const d2u v = *reinterpret_cast<const d2u *>(first + e);
            pre[o][x] = d2{v.x, v.y};
          }
        }
      }
    }
  };
  auto stage = [&](uint32_t mask) {
#pragma unroll
    for (int o = 0; o < 4; o++) {
      if (need(mask, o)) {
#pragma unroll
        for (int x = 0; x < U::NL; x++) {
          const int p = 64 * x + lane;
          if (x < U::NL - 1 || p < U::NP) {
            d2 v = pre[o][x];
            if (x == U::NL - 1 && (U::NV & 1) && p == U::NP - 1) v = d2{v.y, 0.0};
            *reinterpret_cast<d2 *>(&slot[o][2 * p]) = v;
          }
        }
      }
    }
  };

  struct Frag {
    double am[2], ae[2], bm[2], be[2];
  };
  // fragments of k-slice ks (compile-time after unrolling)
  auto frag = [&](int ks) {
    Frag f;
    const bool last = ks == U::NKS - 1;
    const int da = last ? 0 : ao(0, 4 * ks), db = last ? 0 : bo(4 * ks, 0);
#pragma unroll
    for (int r = 0; r < 2; r++) {
      f.am[r] = slot[r][(last ? aml : am0) + da];
      f.ae[r] = slot[r][(last ? ael : ae0) + da];
      f.bm[r] = slot[2 + r][(last ? bml : bm0) + db];
      f.be[r] = slot[2 + r][(last ? bel : be0) + db];
      if (last && U::KT < 4) {
        f.am[r] = kval ? f.am[r] : 0.0;
        f.ae[r] = kval ? f.ae[r] : 0.0;
        f.bm[r] = kval ? f.bm[r] : 0.0;
        f.be[r] = kval ? f.be[r] : 0.0;
      }
    }
    return f;
  };
  // the six MFMAs of result block x = 2r + c at one k-slice
  auto mma = [&](const Frag &f, const double (&aer)[2], const double (&ber)[2], const double (&bes)[2], int x) {
    const int r = x >> 1, c = x & 1;
    acc16[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.am[r], f.bm[c], acc16[x], 0, 0, 0);
    acc4[x][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(f.am[r], f.be[c], acc4[x][0], 0, 0, 0);
    acc4[x][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(f.am[r], ber[c], acc4[x][1], 0, 0, 0);
    acc4[x][2] = __builtin_amdgcn_mfma_f64_4x4x4f64(f.ae[r], f.bm[c], acc4[x][2], 0, 0, 0);
    acc4[x][3] = __builtin_amdgcn_mfma_f64_4x4x4f64(aer[r], f.bm[c], acc4[x][3], 0, 0, 0);
    acc4[x][4] = __builtin_amdgcn_mfma_f64_4x4x4f64(f.ae[r], bes[c], acc4[x][4], 0, 0, 0);
  };
  auto products = [&](uint32_t mine_v) {
    uint32_t mine = (uint32_t)__builtin_amdgcn_readfirstlane((int)mine_v);   // uniform: scalar branches
    Frag fc = frag(0);
#pragma unroll
    for (int ks = 0; ks < U::NKS; ks++) {
      // the product mask stays a scalar register tested per slice, so the
      // branches below are scalar-compare branches, not lane-mask values
      // carried across the slices
      asm volatile("" : "+s"(mine));
      Frag fn;
      if (ks + 1 < U::NKS) fn = frag(ks + 1);
      double aer[2], ber[2], bes[2];
#pragma unroll
      for (int d = 0; d < 2; d++) {
        aer[d] = ror4_f64(fc.ae[d]);
        ber[d] = ror4_f64(fc.be[d]);
        bes[d] = dpp_f64<DPP_ROW_SHR4, 0x6>(fc.be[d]);
      }
#pragma unroll
      for (int x = 0; x < 4; x++)
        if ((mine >> x) & 1u) mma(fc, aer, ber, bes, x);
      if (ks + 1 < U::NKS) fc = fn;
    }
  };

  // step records one at a time (lanes 0..LPR-1 hold one), the record of
  // step s + 2 in flight while step s runs: it has arrived when the blocks
  // of step s + 1 are staged, so decoding never waits for memory
  auto load_rec = [&](int64_t step) { return P.steps[step * SH::LPR + min(lane, SH::LPR - 1)]; };
  int4 rnext = int4{0, 0, 0, 0};
  Rec<SH> R;
  uint32_t mask = 0u;
  if (ns > 0) {
    R.at(load_rec(s0), 0);
    if (ns > 1) rnext = load_rec(s0 + 1);
    mask = R.mask();
    fetch(R, mask);
    stage(mask);
  }
  for (int32_t s = 0; s < ns; s++) {
    const uint32_t cur = mask;
    const bool more = s + 1 < ns;
    if (more) {   // the next step's blocks go in flight
      R.at(rnext, 0);
      if (s + 2 < ns) rnext = load_rec(s0 + s + 2);
      mask = R.mask();
      fetch(R, mask);
    }
    products(cur);
    // this step's fragments were read from LDS before the copies below
    // (one wavefront: LDS operations complete in order)
    if (more) stage(mask);
  }

  // epilogue: C = alpha * acc + beta * C_old, and the Frobenius norm
  const int i4 = lane >> 4, j4 = lane & 3, b4 = (lane >> 2) & 3, lo = b4 & 1;
#pragma unroll
  for (int x = 0; x < 4; x++) {
    const int r = x >> 1, c = x & 1;
    const int32_t cb = sread32(td + 4 + 2 * r + c);
    if (cb < 0) continue;
    const int64_t co = sread64(P.c_off + cb);
    const double *old = nullptr;
    if (P.beta != 0.0 && P.old_blk) {
      const int32_t ob = sread32(P.old_blk + cb);
      if (ob >= 0) old = P.old_val + sread64(P.old_off + ob);
    }
    double ss = 0.0;
    auto put = [&](int row, int col, double v) {
      if (row < S && col < S) {
        double y = P.alpha * v;
        if (old) y += P.beta * old[row + col * S];
        P.c_val[co + row + col * S] = y;
        ss += y * y;
      }
    };
#pragma unroll
    for (int t = 0; t < 4; t++) put(4 * t + kq, i16, acc16[x][t]);
    put(4 * b4 + i4, 16 + 4 * lo + j4, acc4[x][0]);
    put(4 * b4 + i4, 16 + 4 * (lo ^ 1) + j4, acc4[x][1]);
    put(16 + 4 * lo + i4, 4 * b4 + j4, acc4[x][2]);
    put(16 + 4 * (lo ^ 1) + i4, 4 * b4 + j4, acc4[x][3]);
    put(16 + 4 * lo + i4, 16 + 4 * (b4 >> 1) + j4, acc4[x][4]);
    if (P.c_norm) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
      if (lane == 0) P.c_norm[cb] = sqrt(ss);
    }
  }
}

// One workgroup per tile, tiles handed to the XCDs in chunks of `chunk`
// consecutive tiles (the XCDs take chunks in turn).
template <int S, bool TA, bool TB>
__global__ __launch_bounds__(64, 2) void k_tile_uni(TileP P, int64_t ntile, int64_t chunk) {   // two waves per SIMD
  __shared__ __attribute__((aligned(16))) double slot[4][Uni<S>::SLOT];
  const int64_t w = xcd_logical(blockIdx.x, chunk);
  if (w >= ntile) return;   // uniform over the workgroup
  tile_uni<S, TA, TB>(P, w, slot);
}

template <int S, bool TA, bool TB>
void launch_uni_t(const TilePlan &tp, const TileP &p, int64_t max_chunk, hipStream_t s) {
  const XcdMap xm = xcd_map(tp.ntile, max_chunk);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many result tiles for one launch");
  hipLaunchKernelGGL((k_tile_uni<S, TA, TB>), dim3((unsigned)grid), dim3(64), 0, s, p, tp.ntile, xm.chunk);
  HIPCHECK(hipGetLastError());
}

template <int S>
void launch_uni(const TilePlan &tp, const TileP &p, int64_t max_chunk, hipStream_t s) {
  if (p.ta == 0 && p.tb == 0) return launch_uni_t<S, false, false>(tp, p, max_chunk, s);
  if (p.ta == 0 && p.tb == 1) return launch_uni_t<S, false, true>(tp, p, max_chunk, s);
  if (p.ta == 1 && p.tb == 0) return launch_uni_t<S, true, false>(tp, p, max_chunk, s);
  return launch_uni_t<S, true, true>(tp, p, max_chunk, s);
}

// Block sizes with a uniform-size kernel.
#define BSMM_UNI_SIZES(X) X(23)

}  // namespace

bool tile_shape_valid(int ti, int tj) {
  return (ti == 2 && tj == 2) || (ti == 2 && tj == 4) || (ti == 4 && tj == 2) || (ti == 4 && tj == 4) ||
         (ti == 4 && tj == 8) || (ti == 8 && tj == 4);
}

bool tile_uni_size(int32_t sz) {
#define BSMM_UNI_HAS(S) \
  if (sz == S) return true;
  BSMM_UNI_SIZES(BSMM_UNI_HAS)
#undef BSMM_UNI_HAS
  return false;
}

bool tile_path_fits(int32_t nbc, int32_t nbk, TileShape sh) {
  // LDS: the column-group bitmap of a row group, and TI*TJ + 2 k bitmaps per
  // tile wavefront of the step builder
  if (!tile_shape_valid(sh.ti, sh.tj) || nbc < 1 || nbk < 1) return false;
  const size_t w = ((size_t)nbk + 31) / 32;
  const size_t wc = ((size_t)(nbc + sh.tj - 1) / sh.tj + 31) / 32;
  return 4 * w * (size_t)(sh.ti * sh.tj + 2) <= 150 * 1024 && 4 * wc * RG <= 150 * 1024;
}


#define BSMM_TILE_SHAPES(X) X(2, 2) X(2, 4) X(4, 2) X(4, 4) X(4, 8) X(8, 4)

void build_tile_plan(Allocator &al, TileShape sh, const int32_t *ord, const int32_t *crank, const int32_t *cinv,
                     int32_t nbr, int32_t nbc, const int64_t *c_rp, const int32_t *c_ci, const int64_t *seg,
                     const int2 *stack, const OpRows &ar, int32_t nbk, const int32_t *ksz, const int64_t *a_off,
                     const int64_t *b_off, OffsetAreas ob, int64_t *pinned, TilePlan &tp, hipStream_t s) {
  tp.sh = sh;
#define BSMM_BUILD(A, B)                                                                                          \
  if (sh.ti == A && sh.tj == B)                                                                                  \
    return build_plan_t<A, B>(al, ord, crank, cinv, nbr, nbc, c_rp, c_ci, seg, stack, ar, nbk, ksz, a_off, b_off, \
                              ob, pinned, tp, s);
  BSMM_TILE_SHAPES(BSMM_BUILD)
#undef BSMM_BUILD
  fail(BSMM_ERR_INVALID_ARG, "unsupported tile shape");
}

void tile_gemm_launch(const TilePlan &tp, const TileArgs &g, hipStream_t s) {
  if (tp.ntile <= 0) return;
  TileP p;
  p.tiles = tp.tiles.p;
  p.steps = tp.steps.p;
  p.rbs = g.rbs;
  p.cbs = g.cbs;
  p.a_val = g.a_val;
  p.b_val = g.b_val;
  p.a_end = g.a_val + g.a_n;
  p.b_end = g.b_val + g.b_n;
  p.ta = g.ta ? 1 : 0;
  p.tb = g.tb ? 1 : 0;
  p.c_off = g.c_off;
  p.old_blk = g.old_blk;
  p.old_off = g.old_off;
  p.old_val = g.old_val;
  p.c_val = g.c_val;
  p.c_norm = g.c_norm;
  p.alpha = g.alpha;
  p.beta = g.beta;
  const int64_t chunk = g.xcd_chunk > 0 ? g.xcd_chunk : 8192;
  if (g.uni > 0) {
    if (tp.sh.ti != 2 || tp.sh.tj != 2) fail(BSMM_ERR_INVALID_ARG, "the uniform-size kernels take 2 x 2 tiles");
#define BSMM_UNI_GO(S) \
  if (g.uni == S) return launch_uni<S>(tp, p, chunk, s);
    BSMM_UNI_SIZES(BSMM_UNI_GO)
#undef BSMM_UNI_GO
    fail(BSMM_ERR_INVALID_ARG, "no uniform-size kernel for this block size");
  }
#define BSMM_LAUNCH(A, B) \
  if (tp.sh.ti == A && tp.sh.tj == B) return launch_t<A, B>(tp, p, chunk, s);
  BSMM_TILE_SHAPES(BSMM_LAUNCH)
#undef BSMM_LAUNCH
  fail(BSMM_ERR_INVALID_ARG, "unsupported tile shape");
}

}  // namespace bsmm
