// noalloc.hip -- the result-block filter for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops and harnesses
// that forbid hipMalloc).
//
// bsmm_filter drops the blocks whose Frobenius norm is below a threshold
// (the post-multiply filter of arXiv:1705.10218, Section 1) and returns a new
// library-owned matrix; its kernels keep norms, keep flags and scans in
// buffers from the context allocator.  bsmm_filter_noalloc computes the same
// result into caller-owned device buffers, with every intermediate in one
// fixed device array of this file (`scratch`), so it calls no hipMalloc,
// hipFree or host synchronisation.  Each GPU the library runs on holds its
// own copy of the array until the process ends; every call on that GPU
// shares it, so calls that overlap on one GPU race.
//
// Scratch layout (SCRATCH_BYTES in all):
//   keep[NA_MAX_BLOCKS]       uint8  keep flag of every input block
//   rowcnt[2 * NA_MAX_ROWS]   int64  kept blocks and kept values of every row
//   rowval[NA_MAX_ROWS + 1]   int64  first output value of every row
// Every entry a call reads is written earlier in the same call, so nothing
// needs clearing between calls.
#include <mutex>
#include <sstream>
#include <vector>

#include "internal.h"

namespace bsmm {

namespace {

constexpr int64_t NA_MAX_BLOCKS = int64_t(1) << 24;   // 16,777,216 blocks
constexpr int64_t NA_MAX_ROWS = int64_t(1) << 18;     // 262,144 block rows
constexpr size_t KEEP_BYTES = (size_t)NA_MAX_BLOCKS;
constexpr size_t ROWCNT_OFF = KEEP_BYTES;
constexpr size_t ROWVAL_OFF = ROWCNT_OFF + sizeof(int64_t) * 2 * NA_MAX_ROWS;
constexpr size_t SCRATCH_BYTES = ROWVAL_OFF + sizeof(int64_t) * (NA_MAX_ROWS + 1);

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of `scratch` on every device, taken once per device with
// that device current (the host-side name of the array is not a device
// address).
std::mutex g_mu;
std::vector<void *> g_ptr;

// Frobenius norm of one block, 16 lanes: lane g adds the squares of elements
// g, g + 16, ... in ascending order (fused multiply-add), then the 16 partial
// sums combine in a fixed xor tree -- the arithmetic of the block-norm kernel,
// so every keep decision is bitwise the one bsmm_filter takes.
__device__ __forceinline__ double norm16(const double *v, int64_t len, int g) {
  double s = 0.0;
  for (int64_t d = g; d < len; d += 16) s = fma(v[d], v[d], s);
#pragma unroll
  for (int dd = 8; dd >= 1; dd >>= 1) s += __shfl_xor(s, dd, 16);
  return sqrt(s);
}

// One wavefront per block row: its four 16-lane groups take the row's blocks
// in turn, store a keep flag per block (dropped iff norm < eps, so a NaN norm
// keeps its block) and sum the kept blocks and kept values of the row.
__global__ __launch_bounds__(256) void k_na_keep(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                 const int32_t *cbs, const int64_t *off, const double *v,
                                                 int32_t nbr, double eps, unsigned char *keep, int64_t *rowcnt) {
  const int32_t i = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
  if (i >= nbr) return;
  const int lane = threadIdx.x & 63, grp = lane >> 4, g = lane & 15;
  const int64_t m = rbs[i];
  int64_t nb = 0, nv = 0;
  for (int64_t p = rp[i] + grp; p < rp[i + 1]; p += 4) {
    const int64_t o = off[p];
    const double nrm = norm16(v + o, off[p + 1] - o, g);
    const int k = (nrm < eps) ? 0 : 1;
    if (g == 0) {
      keep[p] = (unsigned char)k;
      nb += k;
      nv += k * m * cbs[ci[p]];
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    nb += __shfl_xor(nb, d, 64);
    nv += __shfl_xor(nv, d, 64);
  }
  if (lane == 0) {
    rowcnt[2 * (int64_t)i] = nb;
    rowcnt[2 * (int64_t)i + 1] = nv;
  }
}

// Exclusive scans of the per-row kept blocks (into row_ptr_out) and kept
// values (into rowval), one workgroup: thread t owns a contiguous run of
// rows.  The totals go to counts_out[0..1].
constexpr int NA_SCAN_THREADS = 1024;
__global__ __launch_bounds__(NA_SCAN_THREADS) void k_na_scan(const int64_t *rowcnt, int32_t nbr, int64_t *row_ptr_out,
                                                             int64_t *rowval, int64_t *counts_out) {
  __shared__ int64_t wb[NA_SCAN_THREADS / 64], wv[NA_SCAN_THREADS / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int32_t per = (nbr + NA_SCAN_THREADS - 1) / NA_SCAN_THREADS;
  const int32_t r0 = min(nbr, t * per), r1 = min(nbr, r0 + per);
  int64_t sb = 0, sv = 0;
  for (int32_t r = r0; r < r1; r++) {
    sb += rowcnt[2 * (int64_t)r];
    sv += rowcnt[2 * (int64_t)r + 1];
  }
  int64_t ib = sb, iv = sv;   // inclusive scans over the wavefront
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t ob = __shfl_up(ib, d, 64), ov = __shfl_up(iv, d, 64);
    if (lane >= d) {
      ib += ob;
      iv += ov;
    }
  }
  if (lane == 63) {
    wb[w] = ib;
    wv[w] = iv;
  }
  __syncthreads();
  int64_t bb = ib - sb, bv = iv - sv, tb = 0, tv = 0;
  for (int x = 0; x < NA_SCAN_THREADS / 64; x++) {
    if (x < w) {
      bb += wb[x];
      bv += wv[x];
    }
    tb += wb[x];
    tv += wv[x];
  }
  for (int32_t r = r0; r < r1; r++) {
    row_ptr_out[r] = bb;
    rowval[r] = bv;
    bb += rowcnt[2 * (int64_t)r];
    bv += rowcnt[2 * (int64_t)r + 1];
  }
  if (t == 0) {
    row_ptr_out[nbr] = tb;
    rowval[nbr] = tv;
    counts_out[0] = tb;
    counts_out[1] = tv;
  }
}

// One wavefront per block row: the row's blocks in chunks of 64, lane l
// holding block p = start + l; a ballot prefix places the kept blocks'
// column indices, a wavefront scan of their sizes places their values, and
// the wavefront then copies the kept blocks one after another.
__global__ __launch_bounds__(256) void k_na_compact(const int64_t *rp, const int32_t *ci, const int32_t *rbs,
                                                    const int32_t *cbs, const int64_t *off, const double *v,
                                                    int32_t nbr, const unsigned char *keep,
                                                    const int64_t *row_ptr_out, const int64_t *rowval,
                                                    int32_t *col_idx_out, double *values_out) {
  const int32_t i = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
  if (i >= nbr) return;
  const int lane = threadIdx.x & 63;
  const int64_t m = rbs[i];
  int64_t ob = row_ptr_out[i], ov = rowval[i];
  for (int64_t p0 = rp[i]; p0 < rp[i + 1]; p0 += 64) {
    const int64_t p = p0 + lane;
    const bool in = p < rp[i + 1];
    const bool k = in && keep[p] != 0;
    const int32_t j = in ? ci[p] : 0;
    const int64_t sz = k ? m * cbs[j] : 0;
    const uint64_t bal = __ballot(k);
    const int before = __popcll(bal & ((uint64_t(1) << lane) - 1));
    int64_t inc = sz;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    const int64_t dst = ov + inc - sz;   // first output value of this lane's block
    if (k) col_idx_out[ob + before] = j;
    uint64_t rest = bal;
    while (rest) {
      const int src = __builtin_ctzll(rest);
      rest &= rest - 1;
      const int64_t so = __shfl(in ? off[p] : 0, src, 64);
      const int64_t len = __shfl(sz, src, 64);
      const int64_t d0 = __shfl(dst, src, 64);
      for (int64_t e = lane; e < len; e += 64) values_out[d0 + e] = v[so + e];
    }
    ob += __popcll(bal);
    ov += __shfl(inc, 63, 64);
  }
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
  return x < y + nb && y < x + na;
}

}  // namespace

void noalloc_init(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0) fail(BSMM_ERR_INVALID_ARG, "no such device");
  if ((size_t)device < g_ptr.size() && g_ptr[device]) return;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    std::ostringstream os;
    os << "hipGetSymbolAddress of the filter scratch array failed on device " << device << ": "
       << hipGetErrorString(e);
    fail(BSMM_ERR_DEVICE, os.str());
  }
  if (g_ptr.size() <= (size_t)device) g_ptr.resize((size_t)device + 1, nullptr);
  g_ptr[device] = ptr;
}

}  // namespace bsmm

using namespace bsmm;

extern "C" {

bsmm_status bsmm_filter_noalloc(bsmm_mat m, double eps, int64_t *row_ptr_out, int32_t *col_idx_out,
                                double *values_out, int64_t *counts_out) {
  ABI_BEGIN
  if (!m || !row_ptr_out || !counts_out) fail(BSMM_ERR_INVALID_ARG, "NULL argument");
  if (m->nnzb > 0 && !col_idx_out) fail(BSMM_ERR_INVALID_ARG, "col_idx_out is NULL");
  if (m->n_values > 0 && !values_out) fail(BSMM_ERR_INVALID_ARG, "values_out is NULL");
  if (!(eps >= 0.0)) fail(BSMM_ERR_INVALID_ARG, "eps must be >= 0");
  if (m->nbr > NA_MAX_ROWS || m->nnzb > NA_MAX_BLOCKS) {
    std::ostringstream os;
    os << "bsmm_filter_noalloc takes at most " << NA_MAX_ROWS << " block rows and " << NA_MAX_BLOCKS
       << " blocks (got " << m->nbr << " and " << m->nnzb << ")";
    fail(BSMM_ERR_UNSUPPORTED, os.str());
  }
  const size_t vb = sizeof(double) * (size_t)m->n_values;
  if (overlap(values_out, vb, m->d_values, vb) || overlap(col_idx_out, 4 * (size_t)m->nnzb, m->d_col_idx,
                                                          4 * (size_t)m->nnzb) ||
      overlap(row_ptr_out, 8 * ((size_t)m->nbr + 1), m->d_row_ptr, 8 * ((size_t)m->nbr + 1)))
    fail(BSMM_ERR_ALIAS, "an output buffer overlaps the input matrix");
  bsmm_ctx ctx = m->ctx;
  int prev = -1;
  HIPCHECK(hipGetDevice(&prev));
  if (prev != ctx->device) HIPCHECK(hipSetDevice(ctx->device));
  struct Restore {
    int p, d;
    ~Restore() {
      if (p >= 0 && p != d) (void)hipSetDevice(p);
    }
  } restore{prev, ctx->device};
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((size_t)ctx->device < g_ptr.size()) base = g_ptr[ctx->device];
  }
  if (!base) fail(BSMM_ERR_DEVICE, "filter scratch array not set up on this device");
  unsigned char *keep = static_cast<unsigned char *>(base);
  int64_t *rowcnt = reinterpret_cast<int64_t *>(static_cast<char *>(base) + ROWCNT_OFF);
  int64_t *rowval = reinterpret_cast<int64_t *>(static_cast<char *>(base) + ROWVAL_OFF);
  hipStream_t s = ctx->stream;
  const int32_t nbr = m->nbr;
  const unsigned rows_grid = (unsigned)(((int64_t)nbr * 64 + 255) / 256);
  if (nbr > 0) {
    hipLaunchKernelGGL(k_na_keep, dim3(rows_grid), dim3(256), 0, s, m->d_row_ptr, m->d_col_idx, m->d_rbs, m->d_cbs,
                       m->d_blk_off, m->d_values, nbr, eps, keep, rowcnt);
    HIPCHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_na_scan, dim3(1), dim3(NA_SCAN_THREADS), 0, s, (const int64_t *)rowcnt, nbr, row_ptr_out,
                     rowval, counts_out);
  HIPCHECK(hipGetLastError());
  if (nbr > 0 && m->nnzb > 0) {
    hipLaunchKernelGGL(k_na_compact, dim3(rows_grid), dim3(256), 0, s, m->d_row_ptr, m->d_col_idx, m->d_rbs,
                       m->d_cbs, m->d_blk_off, m->d_values, nbr, (const unsigned char *)keep,
                       (const int64_t *)row_ptr_out, (const int64_t *)rowval, col_idx_out, values_out);
    HIPCHECK(hipGetLastError());
  }
  ABI_END
}

}  // extern "C"
