// gemm_kernels.hip -- batched small-block GEMM on FP64 matrix cores (gfx950).
//
// The local multiplication is a batch of small dense block products summed
// into result blocks (arXiv:1705.10218, Section 2).  One wavefront owns one
// C block for its whole stack segment: the accumulator stays in registers,
// no other wavefront writes that block and no atomics touch C.
//
// Contraction layout.  An MFMA instruction sums four k-slices; its four
// 16-lane k-groups (kq = lane / 16) need not take those slices from the same
// block product -- every product of the segment adds into the same C block.
// So k-group kq walks its own quarter of the segment (products kq, kq+4,
// kq+8, ...) one k at a time, and the MFMA adds the four groups' terms.
// The k padding of a per-product formulation disappears (a 5x5x5 product
// costs 5 k-steps, not 8), and all 16 lanes of a group read one k-column of
// op(A) and one k-row of op(B): contiguous, coalesced loads.  To make both
// contiguous, op(A) blocks are read column-major (m x K, ld m) and op(B)
// blocks row-major (K x n, ld n); a prepass transposes the stored blocks
// whose layout is the other one (A when transa = 'T', B when transb = 'N').
//
// Matrix cores (lane layouts on gfx950, checked on the device):
//   V_MFMA_F64_16X16X4F64: A[i][k] lane i+16k, B[k][j] lane j+16k,
//                          D[i][j] lane j+16(i%4), register i/4.
//     Used when both C edges are in 9..16.
//   V_MFMA_F64_4X4X4F64 (4 blocks b): A_b[i][k] lane i+4b+16k,
//                          B_b[k][j] lane j+4b+16k, D_b[i][j] lane j+4b+16i.
//     Used otherwise: the C block is cut into 4x4 subtiles (MT x NT, even),
//     block b = 2P+Q takes quadrant (P,Q) of the subtile grid and
//     instruction (u,v) subtile (P*MT/2+u, Q*NT/2+v).
// Padded rows / columns are zero-filled, never loaded.
//
// Latency: product parameters (value offsets, k size) for up to 256
// products are staged in LDS per round; operand loads run PF k-steps ahead
// of the matrix core in a register ring.
#include "internal.h"

namespace bsmm {

namespace {

// A work item's descriptor in scalar registers, with its unit bases
// (values into the packed copies; 0 without per-unit addressing).
struct WorkDesc : BlkDesc {
  int64_t ab, bb;
};

struct GemmP {
  const int64_t *a_off;
  const double *a_val;   // op(A) blocks column-major
  const int64_t *b_off;
  const double *b_val;   // op(B) blocks row-major
  const int32_t *c_list;
  const BlkDesc *desc;         // work-item descriptors (quad path)
  const UnitBases *ubase;      // per work item, per-unit addressing only
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
  uint64_t a_len, b_len;       // bytes of the packed copies (BUF path)
  const double *zeros;         // zero page (pointer path)
  uint8_t variant[16];         // kernel variant per (m, n) size class (BUF path)
};

constexpr int ROUND = 256;   // products whose parameters sit in LDS at once
// Wavefronts per workgroup of the GEMM launches: one.  The C blocks of a
// launch take very different times (their stack segments differ by an order
// of magnitude), and a workgroup frees its slot only when its slowest
// wavefront ends; single-wavefront groups keep the SIMDs filled.
constexpr int WPG = 1;
constexpr int PF = 4;        // operand prefetch depth (k-steps)

struct ParamLds {
  int64_t ao[ROUND];
  int64_t bo[ROUND];
  int32_t K[ROUND];
};

// Stage the parameters of products [rb, rb + nr) of the segment in LDS.
__device__ __forceinline__ void load_round(const GemmP &P, ParamLds &pl, int64_t rb, int nr, int m, int lane) {
  for (int q = lane; q < nr; q += 64) {
    const int2 ab = P.stack[rb + q];
    const int64_t ao = P.a_off[ab.x];
    pl.ao[q] = ao;
    pl.K[q] = (int)((P.a_off[ab.x + 1] - ao) / m);
    pl.bo[q] = P.b_off[ab.y];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of k-steps of this round: the longest group's sum of K.
__device__ __forceinline__ int round_steps(const ParamLds &pl, int nr, int lane) {
  int s = 0;
  if (lane < 4)
    for (int t = lane; t < nr; t += 4) s += pl.K[t];
  s = max(s, __shfl_xor(s, 1, 64));
  s = max(s, __shfl_xor(s, 2, 64));
  return __builtin_amdgcn_readfirstlane(s);
}

// Read-after-round fence: the next round rewrites the parameter LDS.
__device__ __forceinline__ void round_end() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------- operand streams
// A lane reads one element per k-step from one row of op(A) (or one column
// of op(B)) of its group's current product, stepping by the leading
// dimension.  BUF: raw buffer loads with a 32-bit byte offset; an offset
// past the buffer end reads 0, which serves padded rows / columns and
// finished groups without any per-step test (arrays below 4 GB).  Otherwise
// 64-bit pointers: finished groups read a zero page, padded rows / columns
// read a clamped (valid) row whose products land only in discarded C
// entries.
constexpr uint32_t OOB = 0xFFFFFFF0u;

template <bool BUF>
struct Stream;

template <>
struct Stream<true> {
  uint32_t off, step;
  __device__ __forceinline__ void set(bool valid, int64_t elem, int ld, const double *, const double *) {
    off = valid ? (uint32_t)(elem * 8) : OOB;
    step = valid ? (uint32_t)(ld * 8) : 0u;
  }
  __device__ __forceinline__ void clear(const double *) {
    off = OOB;
    step = 0u;
  }
  __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, const double *) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  }
  __device__ __forceinline__ void next() { off += step; }
};

template <>
struct Stream<false> {
  const double *p;
  int step;
  // elem is already clamped into the block by the caller
  __device__ __forceinline__ void set(bool active, int64_t elem, int ld, const double *base, const double *zeros) {
    p = active ? base + elem : zeros;
    step = active ? ld : 0;
  }
  __device__ __forceinline__ void clear(const double *zeros) {
    p = zeros;
    step = 0;
  }
  __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t, const double *) const { return *p; }
  __device__ __forceinline__ void next() { p += step; }
};

// Group walker: product t of the round, local k index lk; HA streams of
// op(A) (one per A row the lane feeds) and HB streams of op(B).
template <bool BUF, int HA, int HB>
struct Walker {
  int t, lk, K;
  Stream<BUF> sa[HA], sb[HB];

  __device__ __forceinline__ void open(const GemmP &P, const ParamLds &pl, int nr, int m, int n,
                                       const int (&arow)[HA], const int (&bcol)[HB], const double *zeros) {
    if (t < nr) {
      const int64_t ao = pl.ao[t], bo = pl.bo[t];
      K = pl.K[t];
#pragma unroll
      for (int u = 0; u < HA; u++) {
        if (BUF) sa[u].set(arow[u] < m, ao + arow[u], m, P.a_val, zeros);
        else sa[u].set(true, ao + min(arow[u], m - 1), m, P.a_val, zeros);
      }
#pragma unroll
      for (int v = 0; v < HB; v++) {
        if (BUF) sb[v].set(bcol[v] < n, bo + bcol[v], n, P.b_val, zeros);
        else sb[v].set(true, bo + min(bcol[v], n - 1), n, P.b_val, zeros);
      }
    } else {
      K = 0;
#pragma unroll
      for (int u = 0; u < HA; u++) sa[u].clear(zeros);
#pragma unroll
      for (int v = 0; v < HB; v++) sb[v].clear(zeros);
    }
  }

  __device__ __forceinline__ void start(const GemmP &P, const ParamLds &pl, int kq, int nr, int m, int n,
                                        const int (&arow)[HA], const int (&bcol)[HB], const double *zeros) {
    t = kq;
    lk = 0;
    open(P, pl, nr, m, n, arow, bcol, zeros);
  }

  __device__ __forceinline__ void advance(const GemmP &P, const ParamLds &pl, int nr, int m, int n,
                                          const int (&arow)[HA], const int (&bcol)[HB], const double *zeros) {
    lk++;
    if (lk >= K) {
      if (t < nr) {
        t += 4;
        lk = 0;
        open(P, pl, nr, m, n, arow, bcol, zeros);
      }
    } else {
#pragma unroll
      for (int u = 0; u < HA; u++) sa[u].next();
#pragma unroll
      for (int v = 0; v < HB; v++) sb[v].next();
    }
  }
};

// C = alpha * acc + beta * C_old for one element; sum of squares for the norm.
__device__ __forceinline__ void store_c(const GemmP &P, const double *old, int64_t co, int m, int row, int col,
                                        double v, double &ss) {
  double x = P.alpha * v;
  if (old) x += P.beta * old[row + col * m];
  P.c_val[co + row + (int64_t)col * m] = x;
  ss += x * x;
}

__device__ __forceinline__ const double *old_block(const GemmP &P, int32_t c) {
  if (P.beta != 0.0 && P.old_blk) {
    const int32_t ob = P.old_blk[c];
    if (ob >= 0) return P.old_val + P.old_off[ob];
  }
  return nullptr;
}

__device__ __forceinline__ void store_norm(const GemmP &P, int32_t c, double ss, int lane) {
  if (P.c_norm) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
    if (lane == 0) P.c_norm[c] = sqrt(ss);
  }
}

// ------------------------------------------------------------ 16x16x4 path
typedef double d4 __attribute__((ext_vector_type(4)));

template <bool BUF>
__device__ __forceinline__ void gemm_block_16(const GemmP &P, int32_t c, ParamLds &pl) {
  const int lane = threadIdx.x & 63;
  const int m = P.rbs[P.c_row[c]];
  const int n = P.cbs[P.c_ci[c]];
  const int i16 = lane & 15;
  const int kq = lane >> 4;
  const int arow[1] = {i16}, bcol[1] = {i16};
  const __amdgpu_buffer_rsrc_t ra_ = __builtin_amdgcn_make_buffer_rsrc((void *)P.a_val, (short)0, (int)P.a_len, 0x00020000);
  const __amdgpu_buffer_rsrc_t rb_ = __builtin_amdgcn_make_buffer_rsrc((void *)P.b_val, (short)0, (int)P.b_len, 0x00020000);
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t s0 = P.seg[c], s1 = P.seg[c + 1];
  for (int64_t rb = s0; rb < s1; rb += ROUND) {
    const int nr = (int)min<int64_t>(ROUND, s1 - rb);
    load_round(P, pl, rb, nr, m, lane);
    const int steps = round_steps(pl, nr, lane);
    Walker<BUF, 1, 1> w;
    w.start(P, pl, kq, nr, m, n, arow, bcol, P.zeros);
    double qa[PF], qb[PF];
#pragma unroll
    for (int d = 0; d < PF; d++) {
      qa[d] = w.sa[0].load(ra_, P.a_val);
      qb[d] = w.sb[0].load(rb_, P.b_val);
      w.advance(P, pl, nr, m, n, arow, bcol, P.zeros);
    }
    int s = 0;
    for (; s + PF <= steps; s += PF) {
#pragma unroll
      for (int d = 0; d < PF; d++) {
        const double a = qa[d], b = qb[d];
        qa[d] = w.sa[0].load(ra_, P.a_val);
        qb[d] = w.sb[0].load(rb_, P.b_val);
        w.advance(P, pl, nr, m, n, arow, bcol, P.zeros);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int d = 0; d < PF; d++)
      if (s + d < steps) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[d], qb[d], acc, 0, 0, 0);
    round_end();
  }
  const int64_t co = P.c_off[c];
  const double *old = old_block(P, c);
  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int row = 4 * r + kq;
    if (row < m && i16 < n) store_c(P, old, co, m, row, i16, acc[r], ss);
  }
  store_norm(P, c, ss, lane);
}

// ------------------------------------------------------------- 4x4x4 path
template <bool BUF, int MT, int NT>
__device__ __forceinline__ void gemm_block_44(const GemmP &P, int32_t c, ParamLds &pl) {
  constexpr int HM = MT / 2, HN = NT / 2;
  const int lane = threadIdx.x & 63;
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
  const __amdgpu_buffer_rsrc_t ra_ = __builtin_amdgcn_make_buffer_rsrc((void *)P.a_val, (short)0, (int)P.a_len, 0x00020000);
  const __amdgpu_buffer_rsrc_t rb_ = __builtin_amdgcn_make_buffer_rsrc((void *)P.b_val, (short)0, (int)P.b_len, 0x00020000);
  double acc[HM * HN];
#pragma unroll
  for (int t = 0; t < HM * HN; t++) acc[t] = 0.0;

  const int64_t s0 = P.seg[c], s1 = P.seg[c + 1];
  for (int64_t rb = s0; rb < s1; rb += ROUND) {
    const int nr = (int)min<int64_t>(ROUND, s1 - rb);
    load_round(P, pl, rb, nr, m, lane);
    const int steps = round_steps(pl, nr, lane);
    Walker<BUF, HM, HN> w;
    w.start(P, pl, kq, nr, m, n, arow, bcol, P.zeros);
    double qa[PF][HM], qb[PF][HN];
#pragma unroll
    for (int d = 0; d < PF; d++) {
#pragma unroll
      for (int u = 0; u < HM; u++) qa[d][u] = w.sa[u].load(ra_, P.a_val);
#pragma unroll
      for (int v = 0; v < HN; v++) qb[d][v] = w.sb[v].load(rb_, P.b_val);
      w.advance(P, pl, nr, m, n, arow, bcol, P.zeros);
    }
    int s = 0;
    for (; s + PF <= steps; s += PF) {
#pragma unroll
      for (int d = 0; d < PF; d++) {
        double a[HM], b[HN];
#pragma unroll
        for (int u = 0; u < HM; u++) a[u] = qa[d][u];
#pragma unroll
        for (int v = 0; v < HN; v++) b[v] = qb[d][v];
#pragma unroll
        for (int u = 0; u < HM; u++) qa[d][u] = w.sa[u].load(ra_, P.a_val);
#pragma unroll
        for (int v = 0; v < HN; v++) qb[d][v] = w.sb[v].load(rb_, P.b_val);
        w.advance(P, pl, nr, m, n, arow, bcol, P.zeros);
#pragma unroll
        for (int u = 0; u < HM; u++)
#pragma unroll
          for (int v = 0; v < HN; v++)
            acc[u * HN + v] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u], b[v], acc[u * HN + v], 0, 0, 0);
      }
    }
#pragma unroll
    for (int d = 0; d < PF; d++) {
      if (s + d < steps) {
#pragma unroll
        for (int u = 0; u < HM; u++)
#pragma unroll
          for (int v = 0; v < HN; v++)
            acc[u * HN + v] = __builtin_amdgcn_mfma_f64_4x4x4f64(qa[d][u], qb[d][v], acc[u * HN + v], 0, 0, 0);
      }
    }
    round_end();
  }

  const int64_t co = P.c_off[c];
  const double *old = old_block(P, c);
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < HM; u++) {
    const int row = 4 * (Pq * HM + u) + kq;
#pragma unroll
    for (int v = 0; v < HN; v++)
      if (row < m && bcol[v] < n) store_c(P, old, co, m, row, bcol[v], acc[u * HN + v], ss);
  }
  store_norm(P, c, ss, lane);
}

// ----------------------------------------------------------- quad path
// With the stacks grouped by k size and every equal-k run padded to a
// multiple of 4 entries (null entries), the segment splits into quads of
// four products of one k size; the four k-groups run their quad in lockstep,
// so the k index is uniform.
//
// Operands come from packed copies in k-pair slabs (two consecutive k of
// every row of op(A), or column of op(B), side by side; K padded to even
// with a zero; blocks 16-byte aligned).  One 128-bit load brings a lane two
// k-steps, and the 16 lanes of a k-group read one contiguous run: a buffer
// load costs the address unit about the same for 64 and 128 bits per lane,
// so pairs halve the load-issue time that bounds this kernel.  The slab
// offset rides in the scalar offset (the range check
// covers voffset + soffset + immediate, so a lane whose voffset is out of
// range -- padded row or column, null product -- reads zeros at every k).
// The pad's zero times zero adds an exact 0 when K is odd.  Arrays below
// 2 GB (32-bit offsets with an out-of-range mark that no k offset can wrap).
constexpr uint32_t QOOB = 0x80000000u;

struct QuadLds {
  uint32_t oa[ROUND];   // byte offsets of packed op(A) / op(B) blocks (QOOB = null)
  uint32_t ob[ROUND];
  int32_t Kq[ROUND / 4];
};

// Stack entry q of the round into the parameter LDS.
__device__ __forceinline__ void stage_entry(QuadLds &ql, int q, int2 e) {
  // entries: byte offsets of the two packed blocks with (k - 1) in their low
  // 3 + 2 bits; nulls are QOOB (a quad's first entry is never null)
  const uint32_t oa = (uint32_t)e.x, ob = (uint32_t)e.y;
  ql.oa[q] = oa & ~7u;
  ql.ob[q] = ob & ~7u;
  if ((q & 3) == 0) ql.Kq[q >> 2] = (int)((oa & 7u) | ((ob & 7u) << 3)) + 1;
}

// Entries [from, nr) of the round starting at rb (those below `from` are
// already staged).
__device__ __forceinline__ void load_quads(const GemmP &P, QuadLds &ql, int64_t rb, int nr, int lane, int from = 0) {
  for (int q = from + lane; q < nr; q += 64) stage_entry(ql, q, P.stack[rb + q]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef double d2 __attribute__((ext_vector_type(2)));

// Lane moves inside each 16-lane row (one k-group) of a double, in two
// 32-bit DPP moves; lanes outside BANKS (groups of four lanes) keep x.
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

__device__ __forceinline__ d2 load_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, int soff) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, soff, 0));
}

// SIXTEEN: V_MFMA_F64_16X16X4F64 on MT x NT tiles of 16 (MT, NT in {1, 2});
// otherwise V_MFMA_F64_4X4X4F64 on MT x NT subtiles of 4 (even counts).
// DIAG (one 16x16 tile, both edges at most 8): each 16-lane k-group carries
// two products, lanes 0-7 one and lanes 8-15 another, for rows of op(A) and
// columns of op(B) alike.  One MFMA then sums eight products: the first
// four land in the tile's upper-left 8x8 quadrant, the other four in the
// lower-right one, and the mixed quadrants are discarded.  The segment's
// equal-k runs are padded to groups of eight, so a group of eight products
// shares one k size; the two quadrants are added at the end.
// MIX (edges up to 24, one 16x16 tile plus 4x4 subtiles along an 8-wide
// edge): bit 0 adds rows 16..23, bit 1 columns 16..23.  The edge rows of
// op(A) are loaded once, lane l of a k-group holding row 16 + l % 8 (so
// block b of a V_MFMA_F64_4X4X4F64 sees rows 16 + 4(b%2) ..), and likewise
// the edge columns of op(B).  Per k-slice:
//   rows 0..15 x cols 0..15   one 16x16x4 MFMA;
//   rows 0..15 x cols 16..23  (A rows, B edge) and (A rows, B edge rotated by
//                             four lanes): blocks b take row group b and
//                             column group b%2, then the other one;
//   rows 16..23 x cols 0..15  the same with the roles swapped;
//   rows 16..23 x cols 16..23 (A edge, B edge with lanes 4..11 shifted by
//                             four): block b takes row group b%2 and column
//                             group b/2.
// Four operand loads per k-pair cover 24 x 24, against six for 4x4
// subtiles; the matrix cores do 1 + 5 narrow instructions instead of four
// 16x16 tiles.
// Buffer resource over a packed copy (len bytes) from value offset `base`
// on (uniform): at most 2 GB - 16 bytes, so the null offset QOOB and
// everything past the copy's end read zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t packed_rsrc(const double *v, uint64_t len, int64_t base) {
  const uint64_t rest = len - 8ull * (uint64_t)base;
  const uint32_t ext = rest < 0x7FFFFFF0ull ? (uint32_t)rest : 0x7FFFFFF0u;
  return __builtin_amdgcn_make_buffer_rsrc((void *)(v + base), (short)0, (int)ext, 0x00020000);
}

template <bool SIXTEEN, int MT, int NT, bool DIAG = false, int MIX = 0>
__device__ __forceinline__ void gemm_block_quad(const GemmP &P, const WorkDesc &D, QuadLds &ql, int pre = 0) {
  static_assert(!DIAG || (SIXTEEN && MT == 1 && NT == 1), "diagonal packing uses one 16x16 tile");
  static_assert(MIX == 0 || (SIXTEEN && MT == 1 && NT == 1 && !DIAG), "edge subtiles extend one 16x16 tile");
  constexpr bool XM = (MIX & 1) != 0, XN = (MIX & 2) != 0;
  constexpr int NX = 2 * (int)XM + 2 * (int)XN + (int)(XM && XN);   // 4x4x4 MFMAs per k-slice
  constexpr int G = DIAG ? 8 : 4;   // products per MFMA step
  const int32_t c = D.c;
  constexpr int HM = MIX ? 1 + (int)XM : (SIXTEEN ? MT : MT / 2);
  constexpr int HN = MIX ? 1 + (int)XN : (SIXTEEN ? NT : NT / 2);
  constexpr int T16 = MIX ? 1 : (SIXTEEN ? HM * HN : 1);   // 16x16 accumulators
  // two accumulator sets (the two k-steps of a pair) when a step has a single
  // MFMA chain: a dependent FP64 MFMA waits for the previous result
  constexpr int NC = (HM * HN == 1) ? 2 : 1;
  // pairs in flight: shallower for shapes with many loads per pair, whose
  // ring registers would otherwise cut the wavefronts per SIMD
  constexpr int PF2 = (HM + HN > 3) ? 2 : 3;
  const int lane = threadIdx.x & 63;
  // one C block per wavefront: its sizes are uniform (scalar registers)
  const int m = D.mn & 0xffff;
  const int n = D.mn >> 16;
  const int m16 = 16 * m, n16 = 16 * n;   // bytes of one k-pair slab of op(A) / op(B)
  const int kq = lane >> 4;
  // lane's rows of op(A) / columns of op(B) (-1 if padding)
  int ra[HM], cb[HN];
  // DIAG: which product of the k-group's pair a lane serves
  const int hh = DIAG ? (lane & 15) >> 3 : 0;
  if constexpr (MIX) {
    ra[0] = (lane & 15) < m ? (lane & 15) : -1;
    cb[0] = (lane & 15) < n ? (lane & 15) : -1;
    if constexpr (XM) ra[1] = 16 + (lane & 7) < m ? 16 + (lane & 7) : -1;
    if constexpr (XN) cb[HN - 1] = 16 + (lane & 7) < n ? 16 + (lane & 7) : -1;
  } else if (DIAG) {
    ra[0] = (lane & 7) < m ? (lane & 7) : -1;
    cb[0] = (lane & 7) < n ? (lane & 7) : -1;
  } else if (SIXTEEN) {
#pragma unroll
    for (int u = 0; u < HM; u++) ra[u] = (lane & 15) + 16 * u < m ? (lane & 15) + 16 * u : -1;
#pragma unroll
    for (int v = 0; v < HN; v++) cb[v] = (lane & 15) + 16 * v < n ? (lane & 15) + 16 * v : -1;
  } else {
    const int L4 = lane & 3, bq = (lane >> 2) & 3;
    const int Pq = bq >> 1, Qq = bq & 1;
#pragma unroll
    for (int u = 0; u < HM; u++) {
      const int r = 4 * (Pq * HM + u) + L4;
      ra[u] = r < m ? r : -1;
    }
#pragma unroll
    for (int v = 0; v < HN; v++) {
      const int cc = 4 * (Qq * HN + v) + L4;
      cb[v] = cc < n ? cc : -1;
    }
  }
  const __amdgpu_buffer_rsrc_t rsa = packed_rsrc(P.a_val, P.a_len, D.ab);
  const __amdgpu_buffer_rsrc_t rsb = packed_rsrc(P.b_val, P.b_len, D.bb);
  constexpr int TA = MIX ? (NX > 0 ? NX : 1) : (SIXTEEN ? 1 : HM * HN);   // 4x4 accumulators
  double acc[NC][TA];
  d4 acc16[NC][T16];
#pragma unroll
  for (int h = 0; h < NC; h++) {
#pragma unroll
    for (int t = 0; t < T16; t++) acc16[h][t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < TA; t++) acc[h][t] = 0.0;
  }

  const int64_t s0 = D.s0, s1 = D.s0 + D.ns;
  for (int64_t rbase = s0; rbase < s1; rbase += ROUND) {
    const int nr = (int)min<int64_t>(ROUND, s1 - rbase);   // multiple of G
    const int nq = nr / G;   // product groups of the round
    load_quads(P, ql, rbase, nr, lane, rbase == s0 ? pre : 0);
    // total pairs of the round
    int steps = 0;
    for (int q = lane; q < nq; q += 64) steps += (ql.Kq[q * (G / 4)] + 1) >> 1;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) steps += __shfl_xor(steps, d, 64);
    steps = __builtin_amdgcn_readfirstlane(steps);
    // issue cursor: quad iq, pair ip (uniform), lane offsets of quad iq;
    // the following quad's block offsets and k size are read a quad ahead
    int iq = 0, ip = 0;
    uint32_t va[HM], vb[HN];
    uint32_t noa = QOOB, nob = QOOB;
    int nK = 1 << 20;
    // lane offsets of a quad with block offsets (oa, ob): row r of a slab at
    // 16 r bytes; slab p at p * 16 * (rows) bytes rides in the scalar offset
    auto lane_offsets = [&](uint32_t oa, uint32_t ob, int) {
#pragma unroll
      for (int u = 0; u < HM; u++) va[u] = (ra[u] < 0 || oa == QOOB) ? QOOB : oa + 16u * (uint32_t)ra[u];
#pragma unroll
      for (int v = 0; v < HN; v++) vb[v] = (cb[v] < 0 || ob == QOOB) ? QOOB : ob + 16u * (uint32_t)cb[v];
    };
    int iP;
    const int slot = 4 * hh + kq;   // this lane's product within a group
    {
      const int K0 = __builtin_amdgcn_readfirstlane(ql.Kq[0]);
      iP = (K0 + 1) >> 1;
      lane_offsets(ql.oa[slot], ql.ob[slot], K0);
      if (nq > 1) {
        noa = ql.oa[G + slot];
        nob = ql.ob[G + slot];
        nK = ql.Kq[G / 4];
      }
    }
    d2 qa[PF2][HM], qb[PF2][HN];
    auto issue = [&](d2 (&xa)[HM], d2 (&xb)[HN]) {
      const int sa = ip * m16, sb = ip * n16;
#pragma unroll
      for (int u = 0; u < HM; u++) xa[u] = load_pair(rsa, va[u], sa);
#pragma unroll
      for (int v = 0; v < HN; v++) xb[v] = load_pair(rsb, vb[v], sb);
      if (++ip == iP) {   // uniform: next quad
        ip = 0;
        iq++;
        const int K = __builtin_amdgcn_readfirstlane(nK);
        iP = (K + 1) >> 1;
        lane_offsets(noa, nob, K);
        if (iq + 1 < nq) {
          const int t = G * (iq + 1) + slot;
          noa = ql.oa[t];
          nob = ql.ob[t];
          nK = ql.Kq[(iq + 1) * (G / 4)];
        } else {
          // past the last quad: further issues read zeros (out of range)
          noa = QOOB;
          nob = QOOB;
          nK = 1 << 20;
        }
      }
    };
    auto mma = [&](const d2 (&xa)[HM], const d2 (&xb)[HN]) {
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int h = e % NC;
        if constexpr (MIX) {
          acc16[h][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[0][e], xb[0][e], acc16[h][0], 0, 0, 0);
          int x = 0;
          if constexpr (XN) {
            const double be = xb[HN - 1][e];
            acc[h][x] = __builtin_amdgcn_mfma_f64_4x4x4f64(xa[0][e], be, acc[h][x], 0, 0, 0);
            x++;
            acc[h][x] = __builtin_amdgcn_mfma_f64_4x4x4f64(xa[0][e], dpp_f64<DPP_ROW_ROR4>(be), acc[h][x], 0, 0, 0);
            x++;
          }
          if constexpr (XM) {
            const double ae = xa[1][e];
            acc[h][x] = __builtin_amdgcn_mfma_f64_4x4x4f64(ae, xb[0][e], acc[h][x], 0, 0, 0);
            x++;
            acc[h][x] = __builtin_amdgcn_mfma_f64_4x4x4f64(dpp_f64<DPP_ROW_ROR4>(ae), xb[0][e], acc[h][x], 0, 0, 0);
            x++;
          }
          if constexpr (XM && XN)
            acc[h][x] = __builtin_amdgcn_mfma_f64_4x4x4f64(xa[1][e], dpp_f64<DPP_ROW_SHR4, 0x6>(xb[HN - 1][e]),
                                                           acc[h][x], 0, 0, 0);
        } else if (SIXTEEN) {
#pragma unroll
          for (int u = 0; u < HM; u++)
#pragma unroll
            for (int v = 0; v < HN; v++)
              acc16[h][u * HN + v] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][e], xb[v][e], acc16[h][u * HN + v], 0, 0, 0);
        } else {
#pragma unroll
          for (int u = 0; u < HM; u++)
#pragma unroll
            for (int v = 0; v < HN; v++)
              acc[h][u * HN + v] = __builtin_amdgcn_mfma_f64_4x4x4f64(xa[u][e], xb[v][e], acc[h][u * HN + v], 0, 0, 0);
        }
      }
    };
    // prologue: always PF2 issues (beyond the round they read zeros), so the
    // loop is entered with a fixed number of loads in flight
#pragma unroll
    for (int d = 0; d < PF2; d++) {
      issue(qa[d], qb[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
    // ring: the MFMAs of pair s read slot s % PF2, then the load of pair
    // s + PF2 lands in that same slot (no register copies, so no wait for
    // younger loads)
    int s = 0;
    for (; s + 2 * PF2 <= steps; s += PF2) {   // every issue in range
#pragma unroll
      for (int d = 0; d < PF2; d++) {
        mma(qa[d], qb[d]);
        issue(qa[d], qb[d]);
        __builtin_amdgcn_sched_barrier(0);   // keep the ring order: MFMA(s), load(s + PF2)
      }
    }
    // drain: remaining pairs s .. steps-1, issuing while pairs remain
#pragma unroll
    for (int d = 0; d < 2 * PF2; d++) {
      const int st = s + d;
      if (st < steps) {
        const int slot = d % PF2;
        mma(qa[slot], qb[slot]);
        if (st + PF2 < steps) issue(qa[slot], qb[slot]);
      }
    }
    round_end();
  }

  // fold the accumulator sets in a fixed order
  if constexpr (NC == 2) {
#pragma unroll
    for (int t = 0; t < T16; t++) acc16[0][t] += acc16[NC - 1][t];
#pragma unroll
    for (int t = 0; t < TA; t++) acc[0][t] += acc[NC - 1][t];
  }
  const int64_t co = D.co;
  const double *old = old_block(P, c);
  double ss = 0.0;
  if constexpr (MIX) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = 4 * r + kq, col = lane & 15;
      if (row < m && col < n) store_c(P, old, co, m, row, col, acc16[0][0][r], ss);
    }
    // 4x4x4 results: block b = (lane / 4) % 4, element (lane / 16, lane % 4)
    const int i4 = lane >> 4, j4 = lane & 3, b4 = (lane >> 2) & 3, lo = b4 & 1;
    int x = 0;
    auto put = [&](int row, int col, double v) {
      if (row < m && col < n) store_c(P, old, co, m, row, col, v, ss);
    };
    if constexpr (XN) {
      put(4 * b4 + i4, 16 + 4 * lo + j4, acc[0][x++]);
      put(4 * b4 + i4, 16 + 4 * (lo ^ 1) + j4, acc[0][x++]);
    }
    if constexpr (XM) {
      put(16 + 4 * lo + i4, 4 * b4 + j4, acc[0][x++]);
      put(16 + 4 * (lo ^ 1) + i4, 4 * b4 + j4, acc[0][x++]);
    }
    if constexpr (XM && XN) put(16 + 4 * lo + i4, 16 + 4 * (b4 >> 1) + j4, acc[0][x]);
  } else if (DIAG) {
    // C(i, j) = upper-left (i, j) + lower-right (i + 8, j + 8): the latter
    // sits two registers on and eight lanes over
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const double v = acc16[0][0][r] + __shfl_xor(acc16[0][0][r + 2], 8, 64);
      const int row = 4 * r + kq, col = lane & 15;
      if (row < m && col < n) store_c(P, old, co, m, row, col, v, ss);
    }
  } else if (SIXTEEN) {
#pragma unroll
    for (int u = 0; u < HM; u++)
#pragma unroll
      for (int v = 0; v < HN; v++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = 16 * u + 4 * r + kq, col = 16 * v + (lane & 15);
          if (row < m && col < n) store_c(P, old, co, m, row, col, acc16[0][u * HN + v][r], ss);
        }
  } else {
    const int L4 = lane & 3, bq = (lane >> 2) & 3;
    const int Pq = bq >> 1, Qq = bq & 1;
#pragma unroll
    for (int u = 0; u < HM; u++) {
      const int row = 4 * (Pq * HM + u) + kq;
#pragma unroll
      for (int v = 0; v < HN; v++) {
        const int col = 4 * (Qq * HN + v) + L4;
        if (row < m && col < n) store_c(P, old, co, m, row, col, acc[0][u * HN + v], ss);
      }
    }
  }
  store_norm(P, c, ss, lane);
}

// Size class of a block edge: 4x4 subtiles rounded up to an even count.
__device__ __forceinline__ int edge_tiles(int e) { return ((((e + 3) >> 2) + 1) >> 1) << 1; }

// One launch over all C blocks in the planner's order; every wavefront
// dispatches on its own block's (m, n) class.  Workgroup ids are remapped
// (xcd_logical) so that the 8 XCDs, which the hardware deals ids to
// round-robin, take chunks of 8,192 consecutive work items in turn: each
// chunk keeps its XCD's L2 on a compact region, and the XCDs together stay
// on neighbouring tiles, which their shared infinity cache serves (one
// contiguous stretch per XCD took 11.0 ms on a 4,000-row product, chunks of
// 8,192 10.6 ms, no remap 13.4 ms).
// MAXT bounds the subtile counts compiled in (4: blocks up to 16).
// A work item's descriptor in scalar registers (the index is uniform).
__device__ __forceinline__ WorkDesc load_desc(const GemmP &P, int64_t w) {
  const BlkDesc *d = P.desc + __builtin_amdgcn_readfirstlane((int)w);
  WorkDesc r;
  r.c = __builtin_amdgcn_readfirstlane(d->c);
  r.mn = __builtin_amdgcn_readfirstlane(d->mn);
  r.s0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(d->s0 >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)d->s0);
  r.co = ((int64_t)__builtin_amdgcn_readfirstlane((int)(d->co >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)d->co);
  r.ns = __builtin_amdgcn_readfirstlane(d->ns);
  r.pad = 0;
  r.ab = r.bb = 0;
  if (P.ubase) {   // uniform: per-unit addressing
    const UnitBases *u = P.ubase + __builtin_amdgcn_readfirstlane((int)w);
    r.ab = ((int64_t)__builtin_amdgcn_readfirstlane((int)(u->a >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)u->a);
    r.bb = ((int64_t)__builtin_amdgcn_readfirstlane((int)(u->b >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)u->b);
  }
  return r;
}

// Quad-path dispatch of one C block on its (m, n) class and the class's
// kernel variant.
template <int MAXT>
__device__ __forceinline__ void dispatch_quad(const GemmP &P, const WorkDesc &D, QuadLds &ql, int pre = 0) {
  const int mt = edge_tiles(D.mn & 0xffff);
  const int nt = edge_tiles(D.mn >> 16);
  const int key = mt * 16 + nt;
    // kernel variant of this (m, n) class: 0 = default (16x16 tile when both
    // edges are in 9..16, else 4x4 subtiles), 1 = 16x16 tiles, 2 = 4x4
    // subtiles, 3 = one 16x16 tile packed with two products per k-group
    // (edges up to 8; the stacks were padded to groups of eight for it),
    // 4 = one 16x16 tile plus 4x4 subtiles along the edges beyond 16 (edges
    // in 9..24, one of them above 16)
    const int vid = P.variant[(mt / 2 - 1) * 4 + (nt / 2 - 1)];
    if (vid == 3 && mt == 2 && nt == 2) {
      gemm_block_quad<true, 1, 1, true>(P, D, ql, pre);
      return;
    }
    if constexpr (MAXT > 4) {
      if (vid == 4 && mt >= 4 && nt >= 4 && mt <= 6 && nt <= 6 && (mt == 6 || nt == 6)) {
        if (mt == 6 && nt == 6) gemm_block_quad<true, 1, 1, false, 3>(P, D, ql, pre);
        else if (mt == 6) gemm_block_quad<true, 1, 1, false, 1>(P, D, ql, pre);
        else gemm_block_quad<true, 1, 1, false, 2>(P, D, ql, pre);
        return;
      }
    }
    if (vid == 1 || (vid == 0 && mt == 4 && nt == 4)) {
      const int tm = mt <= 4 ? 1 : 2, tn = nt <= 4 ? 1 : 2;
      if (tm == 1 && tn == 1) {
        gemm_block_quad<true, 1, 1>(P, D, ql, pre);
        return;
      }
      if constexpr (MAXT > 4) {
        if (tm == 1) gemm_block_quad<true, 1, 2>(P, D, ql, pre);
        else if (tn == 1) gemm_block_quad<true, 2, 1>(P, D, ql, pre);
        else gemm_block_quad<true, 2, 2>(P, D, ql, pre);
      }
      return;
    }
    switch (key) {
      case 2 * 16 + 2: gemm_block_quad<false, 2, 2>(P, D, ql, pre); return;
      case 2 * 16 + 4: gemm_block_quad<false, 2, 4>(P, D, ql, pre); return;
      case 4 * 16 + 2: gemm_block_quad<false, 4, 2>(P, D, ql, pre); return;
      case 4 * 16 + 4: gemm_block_quad<false, 4, 4>(P, D, ql, pre); return;
      default: break;
    }
    if constexpr (MAXT > 4) {
      switch (key) {
        case 2 * 16 + 6: gemm_block_quad<false, 2, 6>(P, D, ql, pre); return;
        case 4 * 16 + 6: gemm_block_quad<false, 4, 6>(P, D, ql, pre); return;
        case 6 * 16 + 2: gemm_block_quad<false, 6, 2>(P, D, ql, pre); return;
        case 6 * 16 + 4: gemm_block_quad<false, 6, 4>(P, D, ql, pre); return;
        case 6 * 16 + 6: gemm_block_quad<false, 6, 6>(P, D, ql, pre); return;
        default: break;
      }
    }
    if constexpr (MAXT > 6) {
      switch (key) {
        case 2 * 16 + 8: gemm_block_quad<false, 2, 8>(P, D, ql, pre); return;
        case 4 * 16 + 8: gemm_block_quad<false, 4, 8>(P, D, ql, pre); return;
        case 6 * 16 + 8: gemm_block_quad<false, 6, 8>(P, D, ql, pre); return;
        case 8 * 16 + 2: gemm_block_quad<false, 8, 2>(P, D, ql, pre); return;
        case 8 * 16 + 4: gemm_block_quad<false, 8, 4>(P, D, ql, pre); return;
        case 8 * 16 + 6: gemm_block_quad<false, 8, 6>(P, D, ql, pre); return;
        case 8 * 16 + 8: gemm_block_quad<false, 8, 8>(P, D, ql, pre); return;
        default: break;
      }
    }
}

template <int MAXT, bool BUF>
__global__ __launch_bounds__(64 * WPG) void k_gemm_f64(GemmP P, int64_t nblk, int64_t chunk) {
  __shared__ ParamLds lds[WPG];
  ParamLds &pl = lds[threadIdx.x >> 6];
  QuadLds &ql = *reinterpret_cast<QuadLds *>(&pl);
  const int64_t b = blockIdx.x;
  const int64_t lb = xcd_logical(b, chunk);
  const int64_t w = lb * WPG + (threadIdx.x >> 6);
  if (w >= nblk) return;   // uniform per wavefront
  if constexpr (BUF) {
    const WorkDesc D = load_desc(P, w);
    dispatch_quad<MAXT>(P, D, ql);
    return;
  } else {
  const int32_t c = __builtin_amdgcn_readfirstlane(P.c_list ? P.c_list[w] : (int32_t)w);
  const int mt = edge_tiles(P.rbs[P.c_row[c]]);
  const int nt = edge_tiles(P.cbs[P.c_ci[c]]);
  const int key = mt * 16 + nt;
  switch (key) {
    case 2 * 16 + 2: gemm_block_44<BUF, 2, 2>(P, c, pl); break;
    case 2 * 16 + 4: gemm_block_44<BUF, 2, 4>(P, c, pl); break;
    case 4 * 16 + 2: gemm_block_44<BUF, 4, 2>(P, c, pl); break;
    case 4 * 16 + 4: gemm_block_16<BUF>(P, c, pl); break;
    default:
      if constexpr (MAXT > 4) {
        switch (key) {
          case 2 * 16 + 6: gemm_block_44<BUF, 2, 6>(P, c, pl); break;
          case 2 * 16 + 8: gemm_block_44<BUF, 2, 8>(P, c, pl); break;
          case 4 * 16 + 6: gemm_block_44<BUF, 4, 6>(P, c, pl); break;
          case 4 * 16 + 8: gemm_block_44<BUF, 4, 8>(P, c, pl); break;
          case 6 * 16 + 2: gemm_block_44<BUF, 6, 2>(P, c, pl); break;
          case 6 * 16 + 4: gemm_block_44<BUF, 6, 4>(P, c, pl); break;
          case 6 * 16 + 6: gemm_block_44<BUF, 6, 6>(P, c, pl); break;
          case 6 * 16 + 8: gemm_block_44<BUF, 6, 8>(P, c, pl); break;
          case 8 * 16 + 2: gemm_block_44<BUF, 8, 2>(P, c, pl); break;
          case 8 * 16 + 4: gemm_block_44<BUF, 8, 4>(P, c, pl); break;
          case 8 * 16 + 6: gemm_block_44<BUF, 8, 6>(P, c, pl); break;
          case 8 * 16 + 8: gemm_block_44<BUF, 8, 8>(P, c, pl); break;
          default: break;
        }
      }
      break;
  }
  }
}

// Several multiplications in one launch: wavefront w takes C block
// w - start[r] of request r (start: prefix of the requests' C block counts),
// with request r's parameters.  Every request's C blocks are computed exactly
// as in a launch of its own, so its results are bitwise the same.
template <int MAXT>
__global__ __launch_bounds__(64 * WPG) void k_gemm_f64_multi(const GemmP *ps, const int64_t *start, int nreq,
                                                        int64_t nblk, int64_t chunk) {
  __shared__ ParamLds lds[WPG];
  ParamLds &pl = lds[threadIdx.x >> 6];
  QuadLds &ql = *reinterpret_cast<QuadLds *>(&pl);
  const int64_t b = blockIdx.x;
  const int64_t lb = xcd_logical(b, chunk);
  const int64_t w = lb * WPG + (threadIdx.x >> 6);
  if (w >= nblk) return;   // uniform per wavefront
  int r = 0;
  while (r + 1 < nreq && start[r + 1] <= w) r++;
  r = __builtin_amdgcn_readfirstlane(r);
  const GemmP &P = ps[r];
  const int64_t lw = w - start[r];
  const WorkDesc D = load_desc(P, lw);
  dispatch_quad<MAXT>(P, D, ql);
}

// Work list: tiles of `tr` consecutive rows of the locality order; inside a
// tile, C blocks go column by column, the columns in the same locality order
// (rank[j] = position of column j in it).  A block B(k,j) feeds only the C
// blocks of column j, one per row i with A(i,k) stored, so running a
// column's blocks of neighbouring rows back to back keeps B(k,j) in L2;
// neighbouring columns need neighbouring k, so the tile's A(i,k) in use at
// any time are a compact subset as well.
__global__ void k_order_counts(const int32_t *ord, const int64_t *c_rp, int32_t nbr, int32_t tr, int64_t *cnt) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;   // tile
  const int32_t ntile = (nbr + tr - 1) / tr;
  if (t >= ntile) return;
  int64_t s = 0;
  for (int32_t r = t * tr; r < min(nbr, (t + 1) * tr); r++) s += c_rp[ord[r] + 1] - c_rp[ord[r]];
  cnt[t] = s;
}

// One workgroup per tile: counting sort of the tile's C blocks by column
// (LDS histogram over nbc columns); ties in a column fall in any order.
__global__ __launch_bounds__(256) void k_order_fill(const int32_t *ord, const int32_t *rank, const int64_t *c_rp,
                                                    const int32_t *c_ci, int32_t nbr, int32_t nbc, int32_t tr,
                                                    const int64_t *start, int32_t *c_list) {
  extern __shared__ int32_t hist[];   // nbc counters, then the scan
  __shared__ int32_t wsum[4];
  const int32_t t = blockIdx.x;
  const int32_t r0 = t * tr, r1 = min(nbr, r0 + tr);
  if (nbc == 0) {   // no column histogram: the tile's rows one after another
    int64_t off = start[t];
    for (int32_t r = r0; r < r1; r++) {
      const int64_t c0 = c_rp[ord[r]], len = c_rp[ord[r] + 1] - c0;
      for (int64_t q = threadIdx.x; q < len; q += blockDim.x) c_list[off + q] = (int32_t)(c0 + q);
      off += len;
    }
    return;
  }
  for (int32_t j = threadIdx.x; j < nbc; j += blockDim.x) hist[j] = 0;
  __syncthreads();
  for (int32_t r = r0; r < r1; r++) {
    const int64_t c0 = c_rp[ord[r]], c1 = c_rp[ord[r] + 1];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) atomicAdd(&hist[rank ? rank[c_ci[c]] : c_ci[c]], 1);
  }
  __syncthreads();
  // exclusive scan of hist over nbc entries (each thread a contiguous chunk)
  const int32_t per = (nbc + blockDim.x - 1) / blockDim.x;
  const int32_t j0 = threadIdx.x * per, j1 = min(nbc, j0 + per);
  int32_t loc = 0;
  for (int32_t j = j0; j < j1; j++) loc += hist[j];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t run = inc - loc;
  for (int w = 0; w < wv; w++) run += wsum[w];
  for (int32_t j = j0; j < j1; j++) {
    const int32_t h = hist[j];
    hist[j] = run;
    run += h;
  }
  __syncthreads();
  const int64_t o = start[t];
  for (int32_t r = r0; r < r1; r++) {
    const int64_t c0 = c_rp[ord[r]], c1 = c_rp[ord[r] + 1];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
      const int32_t at = atomicAdd(&hist[rank ? rank[c_ci[c]] : c_ci[c]], 1);
      c_list[o + at] = (int32_t)c;
    }
  }
}

// ---------------------------------------------------------------- prepass
// Transpose every stored block of a matrix (column-major r x c becomes
// column-major c x r, same offsets).  One workgroup per block row.
__global__ __launch_bounds__(256) void k_transpose_blocks(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                          const int32_t *cbs, const int64_t *off, const double *in,
                                                          double *out) {
  const int32_t i = blockIdx.x;
  const int r = rbs[i];
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const int cc = cbs[ci[p]];
    const int64_t o = off[p];
    const int len = r * cc;
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
      const int a = e % r, b = e / r;   // element (a, b) of the r x cc block
      out[o + b + (int64_t)a * cc] = in[o + e];
    }
  }
}

// Workgroup ids are remapped as in the GEMM (each XCD a contiguous stretch
// of the work list): the C blocks of a stretch lie in few row tiles, so
// each XCD's L2 holds the index data of its own tiles only.
__global__ void k_build_desc(int64_t n, const int32_t *c_list, const int32_t *c_row, const int32_t *c_ci,
                             const int32_t *rbs, const int32_t *cbs, const int64_t *seg, const int64_t *c_off,
                             DescBases bases, BlkDesc *desc, int64_t per_xcd) {
  const int64_t b = blockIdx.x;
  const int64_t w = ((b & 7) * per_xcd + (b >> 3)) * blockDim.x + threadIdx.x;
  if (w >= n) return;
  const int32_t c = c_list ? c_list[w] : (int32_t)w;
  BlkDesc d;
  d.c = c;
  d.mn = rbs[c_row[c]] | (cbs[c_ci[c]] << 16);
  d.s0 = seg[c];
  d.ns = (int32_t)(seg[c + 1] - seg[c]);
  d.co = c_off[c];
  d.pad = 0;
  desc[w] = d;
  if (bases.out) bases.out[w] = UnitBases{bases.a[c_row[c]], bases.b[c_ci[c]]};
}

}  // namespace

void build_desc(int64_t n, const int32_t *c_list, const int32_t *c_row, const int32_t *c_ci, const int32_t *rbs,
                const int32_t *cbs, const int64_t *seg, const int64_t *c_off, DescBases bases, BlkDesc *desc,
                hipStream_t s) {
  if (n <= 0) return;
  const int64_t per_xcd = ((n + 255) / 256 + 7) / 8;
  hipLaunchKernelGGL(k_build_desc, dim3((unsigned)(per_xcd * 8)), dim3(256), 0, s, n, c_list, c_row, c_ci, rbs, cbs,
                     seg, c_off, bases, desc, per_xcd);
  HIPCHECK(hipGetLastError());
}

void transpose_blocks(const bsmm_mat_s &x, double *out, hipStream_t s) {
  if (x.nbr == 0 || x.nnzb == 0) return;
  hipLaunchKernelGGL(k_transpose_blocks, dim3(x.nbr), dim3(256), 0, s, x.d_row_ptr, x.d_col_idx, x.d_rbs, x.d_cbs,
                     x.d_blk_off, x.d_values, out);
  HIPCHECK(hipGetLastError());
}

void build_work_list(Allocator &al, const int32_t *d_ord, const int32_t *d_rank, const int64_t *c_rp,
                     const int32_t *c_ci, int32_t nbr, int32_t nbc, int32_t tile_rows, int32_t *c_list, hipStream_t s) {
  if (nbr == 0) return;
  const int32_t tr = std::max(tile_rows, 1);
  const int32_t ntile = (nbr + tr - 1) / tr;
  DBuf<int64_t> cnt(al, ntile), start(al, (size_t)ntile + 1);
  hipLaunchKernelGGL(k_order_counts, dim3((ntile + 255) / 256), dim3(256), 0, s, d_ord, c_rp, nbr, tr, cnt.p);
  HIPCHECK(hipGetLastError());
  exclusive_scan_i64(al, cnt.p, start.p, ntile, s);
  const size_t lds = sizeof(int32_t) * (size_t)std::max(nbc, 1);
  if (lds > 65536)
    HIPCHECK(hipFuncSetAttribute((const void *)k_order_fill, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_order_fill, dim3(ntile), dim3(256), lds, s, d_ord, d_rank, c_rp, c_ci, nbr, nbc, tr,
                     (const int64_t *)start.p, c_list);
  HIPCHECK(hipGetLastError());
}

static GemmP make_params(const GemmArgs &g) {
  GemmP p;
  p.a_off = g.a->blk_off;
  p.a_val = g.a_cm;
  p.b_off = g.b->blk_off;
  p.b_val = g.b_rm;
  p.c_list = g.c_list;
  p.desc = g.desc;
  p.ubase = g.ubase;
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
  const bool buf = g.quads;
  if (buf) {   // quad path: packed copies (op(A) row-major, op(B) column-major, k padded to even)
    p.a_val = g.a_pack;
    p.b_val = g.b_pack;
  }
  p.a_len = buf ? g.a_bytes : 0u;
  p.b_len = buf ? g.b_bytes : 0u;
  p.zeros = g.zeros;
  for (int t = 0; t < 16; t++) p.variant[t] = g.variant[t];
  return p;
}

void gemm_launch(const GemmArgs &g, int64_t nnzb_c, int max_edge, hipStream_t s) {
  if (nnzb_c <= 0) return;
  if (max_edge > 32) fail(BSMM_ERR_UNSUPPORTED, "block size above 32");
  const GemmP p = make_params(g);
  const bool buf = g.quads;
  const int64_t nwg = (nnzb_c + WPG - 1) / WPG;
  const XcdMap xm = xcd_map(nwg);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many C blocks for one launch");
  if (max_edge <= 16 && buf)
    hipLaunchKernelGGL((k_gemm_f64<4, true>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else if (max_edge <= 24 && buf)   // shapes up to 24: the register budget of the 24-wide shapes
    hipLaunchKernelGGL((k_gemm_f64<6, true>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else if (max_edge <= 16)
    hipLaunchKernelGGL((k_gemm_f64<4, false>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else if (buf)
    hipLaunchKernelGGL((k_gemm_f64<8, true>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  else
    hipLaunchKernelGGL((k_gemm_f64<8, false>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, p, nnzb_c, xm.chunk);
  HIPCHECK(hipGetLastError());
}

size_t gemm_multi_stage_bytes(int n) { return sizeof(GemmP) * (size_t)n + sizeof(int64_t) * ((size_t)n + 1); }

void gemm_launch_multi(Allocator &al, const std::vector<const GemmArgs *> &gs, const std::vector<int64_t> &nnzb,
                       int max_edge, void *h_stage, size_t stage_bytes, void *d_stage, hipStream_t s) {
  const int n = (int)gs.size();
  if (n == 0) return;
  if (max_edge > 32) fail(BSMM_ERR_UNSUPPORTED, "block size above 32");
  const size_t need = sizeof(GemmP) * n + sizeof(int64_t) * (n + 1);
  if (need > stage_bytes) fail(BSMM_ERR_UNSUPPORTED, "too many requests in one batch");
  GemmP *hp = static_cast<GemmP *>(h_stage);
  int64_t *hs = reinterpret_cast<int64_t *>(static_cast<char *>(h_stage) + sizeof(GemmP) * n);
  hs[0] = 0;
  for (int r = 0; r < n; r++) {
    if (!gs[r]->quads) fail(BSMM_ERR_UNSUPPORTED, "batched execution needs the packed-operand path");
    hp[r] = make_params(*gs[r]);
    hs[r + 1] = hs[r] + std::max<int64_t>(nnzb[r], 0);
  }
  const int64_t total = hs[n];
  if (total == 0) return;
  HIPCHECK(hipMemcpyAsync(d_stage, h_stage, need, hipMemcpyHostToDevice, s));
  const GemmP *dp = static_cast<const GemmP *>(d_stage);
  const int64_t *ds = reinterpret_cast<const int64_t *>(static_cast<const char *>(d_stage) + sizeof(GemmP) * n);
  const int64_t nwg = (total + WPG - 1) / WPG;
  const XcdMap xm = xcd_map(nwg);
  const int64_t grid = xm.per_xcd * 8;
  if (grid > INT32_MAX) fail(BSMM_ERR_UNSUPPORTED, "too many C blocks for one launch");
  if (max_edge <= 16)
    hipLaunchKernelGGL((k_gemm_f64_multi<4>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, dp, ds, n, total, xm.chunk);
  else if (max_edge <= 24)
    hipLaunchKernelGGL((k_gemm_f64_multi<6>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, dp, ds, n, total, xm.chunk);
  else
    hipLaunchKernelGGL((k_gemm_f64_multi<8>), dim3((unsigned)grid), dim3(64 * WPG), 0, s, dp, ds, n, total, xm.chunk);
  HIPCHECK(hipGetLastError());
  (void)al;
}

}  // namespace bsmm
