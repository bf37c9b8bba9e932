/*
 * oracle.c -- plain CPU FP64 reference for the local block-sparse multiply
 *             C = alpha * op(A) * op(B) + beta * C_old  (with norm filtering).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header or table with the GPU library, and the
 * product path never calls it.
 *
 * What it follows (arXiv:1705.10218, Lazzaro et al., PASC'17):
 *   - Section 2 (DBCSR library): matrices are stored in blocked CSR form; the
 *     elements are grouped into dense blocks whose row/column sizes come from
 *     the atomic basis; the result pattern is not fixed in advance but comes
 *     out of the product, with blocks below a threshold skipped during the
 *     multiplication or removed after it.
 *   - Section 2, local multiplication: the product is a sum of small dense
 *     block products; a block product is performed only when the product of
 *     the two block norms passes the threshold (on-the-fly filter).
 *   - Section 1: filtering happens in two phases, on the fly and after each
 *     multiplication.
 *   - Related work: the row-by-row serial sparse product of Gustavson is the
 *     classic algorithm; this oracle is that algorithm at block granularity.
 *
 * Readings taken where the paper is silent:
 *   R1 norm = Frobenius norm, FP64, for both filter phases;
 *   R2 a block product is kept iff normA*normB >= eps, and a result block is
 *      kept iff its norm >= eps (so eps = 0 filters nothing);
 *   R3 eps is not scaled by alpha or by the number of terms;
 *   R4 the same eps is used by both phases;
 *   R5 retain_sparsity: the result pattern is exactly the pattern of C_old;
 *      products landing outside it are discarded and no post-filter runs;
 *   R6 beta == 0: C_old is not read (BLAS convention);
 *   R7 alpha is applied once to the accumulated sum: c = alpha*acc + beta*c_old;
 *   R8 blocks are column-major (leading dimension = block row count), block
 *      column indices are strictly increasing inside a block row.
 *
 * Arithmetic: every product block accumulates with a plain triple loop in
 * ascending k-block order and ascending inner index (so an element is the
 * sequential dot product over the kept terms in ascending global index
 * order).  Compiled with -O2 -ffp-contract=off: no fused multiply-add, no
 * reassociation.  Threads split block rows only, so the result is bitwise
 * independent of the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- matrices */

typedef struct {
  int32_t nbr, nbc;        /* block rows / block columns                      */
  int32_t *rbs, *cbs;      /* row / column block sizes                        */
  int64_t nnzb;            /* stored blocks                                    */
  int64_t *row_ptr;        /* nbr+1                                            */
  int32_t *col_idx;        /* nnzb, strictly increasing inside a row          */
  int64_t *off;            /* nnzb+1 element offsets of the blocks            */
  double *val;             /* off[nnzb] values, blocks column-major           */
  int own;                 /* 1 if the arrays above were malloc'ed here        */
} omat;

typedef struct {
  int32_t nbr, nbc;
  int32_t *rbs, *cbs;
  int64_t nnzb;
  int64_t *row_ptr;
  int32_t *col_idx;
  double *val;
  int64_t n_val;
  int64_t n_products;      /* block products actually multiplied             */
  int64_t n_candidates;    /* block products before the on-the-fly filter    */
  double useful_flops;     /* sum over kept products of 2*m*k*n              */
} oracle_result;

static void omat_free(omat *m) {
  if (!m->own) return;
  free(m->rbs); free(m->cbs); free(m->row_ptr); free(m->col_idx);
  free(m->off); free(m->val);
}

static int64_t *block_offsets(int32_t nbr, const int32_t *rbs, const int32_t *cbs,
                              const int64_t *row_ptr, const int32_t *col_idx) {
  int64_t nnzb = row_ptr[nbr];
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzb + 1));
  int64_t o = 0;
  for (int32_t i = 0; i < nbr; i++)
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      off[p] = o;
      o += (int64_t)rbs[i] * cbs[col_idx[p]];
    }
  off[nnzb] = o;
  return off;
}

/* Wrap caller arrays (no copy) as an omat. */
static omat wrap(int32_t nbr, int32_t nbc, const int32_t *rbs, const int32_t *cbs,
                 const int64_t *row_ptr, const int32_t *col_idx, const double *val) {
  omat m;
  m.nbr = nbr; m.nbc = nbc;
  m.rbs = (int32_t *)rbs; m.cbs = (int32_t *)cbs;
  m.row_ptr = (int64_t *)row_ptr; m.col_idx = (int32_t *)col_idx;
  m.nnzb = row_ptr[nbr];
  m.off = block_offsets(nbr, rbs, cbs, row_ptr, col_idx);
  m.val = (double *)val;
  m.own = 0;
  return m;
}

/* Transpose: the block grid is transposed and so is every block.  Block
 * (i,j) of size m x n becomes block (j,i) of size n x m with element (c,r)
 * equal to the old element (r,c).  Entries of a new row are produced in
 * ascending old-row order, i.e. sorted. */
static omat transpose(const omat *x) {
  omat t;
  t.nbr = x->nbc; t.nbc = x->nbr; t.nnzb = x->nnzb; t.own = 1;
  t.rbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t.nbr ? t.nbr : 1));
  t.cbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t.nbc ? t.nbc : 1));
  memcpy(t.rbs, x->cbs, sizeof(int32_t) * (size_t)t.nbr);
  memcpy(t.cbs, x->rbs, sizeof(int32_t) * (size_t)t.nbc);
  t.row_ptr = (int64_t *)calloc((size_t)t.nbr + 1, sizeof(int64_t));
  t.col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t.nnzb ? t.nnzb : 1));
  int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (size_t)(t.nnzb ? t.nnzb : 1));
  for (int64_t p = 0; p < x->nnzb; p++) t.row_ptr[x->col_idx[p] + 1]++;
  for (int32_t r = 0; r < t.nbr; r++) t.row_ptr[r + 1] += t.row_ptr[r];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(t.nbr ? t.nbr : 1));
  for (int32_t r = 0; r < t.nbr; r++) fill[r] = t.row_ptr[r];
  for (int32_t i = 0; i < x->nbr; i++)
    for (int64_t p = x->row_ptr[i]; p < x->row_ptr[i + 1]; p++) {
      int32_t j = x->col_idx[p];
      int64_t q = fill[j]++;
      t.col_idx[q] = i;
      src[q] = p;
    }
  free(fill);
  t.off = block_offsets(t.nbr, t.rbs, t.cbs, t.row_ptr, t.col_idx);
  t.val = (double *)malloc(sizeof(double) * (size_t)(t.off[t.nnzb] ? t.off[t.nnzb] : 1));
  for (int32_t r = 0; r < t.nbr; r++)
    for (int64_t q = t.row_ptr[r]; q < t.row_ptr[r + 1]; q++) {
      int64_t p = src[q];
      int32_t m = x->rbs[t.col_idx[q]];   /* old block rows    */
      int32_t n = x->cbs[r];              /* old block columns */
      const double *a = x->val + x->off[p];
      double *b = t.val + t.off[q];
      for (int32_t c = 0; c < n; c++)
        for (int32_t rr = 0; rr < m; rr++) b[c + (int64_t)rr * n] = a[rr + (int64_t)c * m];
    }
  free(src);
  return t;
}

/* Frobenius norm of one block: square root of the sequential sum of squares
 * taken in storage order. */
static double block_norm(const double *v, int64_t len) {
  double s = 0.0;
  for (int64_t e = 0; e < len; e++) s += v[e] * v[e];
  return sqrt(s);
}

static void all_norms(const omat *x, double *out) {
  for (int64_t p = 0; p < x->nnzb; p++) out[p] = block_norm(x->val + x->off[p], x->off[p + 1] - x->off[p]);
}

/* ------------------------------------------------------------ row results */

typedef struct {
  int64_t nb;         /* blocks in this result row  */
  int32_t *cols;
  double *val;        /* concatenated blocks        */
  int64_t nval;
  int64_t n_products, n_candidates;
  double flops;
} row_out;

typedef struct {
  const omat *a, *b, *cold;
  const double *na, *nb;
  double alpha, beta, eps;
  int retain;
  int has_cold;        /* C_old is present (needed when beta != 0 or retain) */
  row_out *rows;
  const int32_t *sel;  /* rows to compute (NULL = all rows)       */
  int64_t n_sel;
  int64_t next;        /* shared work counter over rows or sel   */
  pthread_mutex_t lock;
} mul_job;

static int32_t find_col(const int32_t *cols, int64_t lo, int64_t hi, int32_t j) {
  /* index of j in the sorted slice cols[lo,hi), or -1 */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (cols[mid] == j) return (int32_t)(mid);
    if (cols[mid] < j) lo = mid + 1; else hi = mid;
  }
  return -1;
}

static void do_row(mul_job *J, int32_t i, double **acc, int32_t *touched) {
  const omat *A = J->a, *B = J->b, *C0 = J->cold;
  int32_t m = A->rbs[i];
  int64_t ntouch = 0;
  row_out *R = &J->rows[i];
  memset(R, 0, sizeof(*R));
  /* Gustavson: for each stored A(i,k), ascending k, and each stored B(k,j),
   * ascending j, add A(i,k) B(k,j) into the accumulator of C(i,j). */
  for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) {
    int32_t k = A->col_idx[p];
    int32_t kk = A->cbs[k];
    const double *ablk = A->val + A->off[p];
    for (int64_t q = B->row_ptr[k]; q < B->row_ptr[k + 1]; q++) {
      int32_t j = B->col_idx[q];
      int32_t n = B->cbs[j];
      R->n_candidates++;
      if (J->retain && find_col(C0->col_idx, C0->row_ptr[i], C0->row_ptr[i + 1], j) < 0) continue;
      if (J->na[p] * J->nb[q] < J->eps) continue;   /* R2: keep iff >= eps */
      if (!acc[j]) {
        acc[j] = (double *)calloc((size_t)m * n, sizeof(double));
        touched[ntouch++] = j;
      }
      double *c = acc[j];
      const double *bblk = B->val + B->off[q];
      for (int32_t cc = 0; cc < n; cc++)
        for (int32_t r = 0; r < m; r++) {
          double s = c[r + (int64_t)cc * m];
          for (int32_t l = 0; l < kk; l++) s += ablk[r + (int64_t)l * m] * bblk[l + (int64_t)cc * kk];
          c[r + (int64_t)cc * m] = s;
        }
      R->n_products++;
      R->flops += 2.0 * m * kk * n;
    }
  }
  /* Result pattern of this row: the touched columns, plus C_old's columns
   * when beta != 0; exactly C_old's columns under retain_sparsity. */
  int32_t nbc = B->nbc;
  char *inrow = (char *)calloc((size_t)(nbc ? nbc : 1), 1);
  if (J->retain) {
    for (int64_t q = C0->row_ptr[i]; q < C0->row_ptr[i + 1]; q++) inrow[C0->col_idx[q]] = 1;
  } else {
    for (int64_t t = 0; t < ntouch; t++) inrow[touched[t]] = 1;
    if (J->beta != 0.0 && J->has_cold)
      for (int64_t q = C0->row_ptr[i]; q < C0->row_ptr[i + 1]; q++) inrow[C0->col_idx[q]] = 1;
  }
  int64_t cnt = 0, nval = 0;
  for (int32_t j = 0; j < nbc; j++)
    if (inrow[j]) { cnt++; nval += (int64_t)m * B->cbs[j]; }
  int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt ? cnt : 1));
  double *val = (double *)malloc(sizeof(double) * (size_t)(nval ? nval : 1));
  int64_t nb = 0, o = 0;
  for (int32_t j = 0; j < nbc; j++) {
    if (!inrow[j]) continue;
    int32_t n = B->cbs[j];
    int64_t len = (int64_t)m * n;
    const double *old = NULL;
    if (J->beta != 0.0 && J->has_cold) {
      int32_t q = find_col(C0->col_idx, C0->row_ptr[i], C0->row_ptr[i + 1], j);
      if (q >= 0) old = C0->val + C0->off[q];
    }
    double *dst = val + o;
    for (int64_t e = 0; e < len; e++) {
      double v = acc[j] ? J->alpha * acc[j][e] : 0.0;   /* R7 */
      if (old) v = v + J->beta * old[e];               /* R6: beta==0 never reads */
      dst[e] = v;
    }
    /* post-filter (R2, R5): drop result blocks whose norm is below eps */
    if (!J->retain && block_norm(dst, len) < J->eps) continue;
    cols[nb++] = j;
    o += len;
  }
  R->nb = nb; R->cols = cols; R->val = val; R->nval = o;
  for (int64_t t = 0; t < ntouch; t++) { free(acc[touched[t]]); acc[touched[t]] = NULL; }
  free(inrow);
}

static void *worker(void *arg) {
  mul_job *J = (mul_job *)arg;
  int32_t nbc = J->b->nbc;
  double **acc = (double **)calloc((size_t)(nbc ? nbc : 1), sizeof(double *));
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nbc ? nbc : 1));
  int64_t total = J->sel ? J->n_sel : J->a->nbr;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t t = J->next++;
    pthread_mutex_unlock(&J->lock);
    if (t >= total) break;
    int32_t i = J->sel ? J->sel[t] : (int32_t)t;
    do_row(J, i, acc, touched);
  }
  free(acc); free(touched);
  return NULL;
}

/* ------------------------------------------------------------ entry points */

/* Frobenius norm of every stored block, in storage (CSR) order. */
int oracle_block_norms(int32_t nbr, int32_t nbc, const int32_t *rbs, const int32_t *cbs,
                       const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                       double *out) {
  omat x = wrap(nbr, nbc, rbs, cbs, row_ptr, col_idx, val);
  all_norms(&x, out);
  free(x.off);
  return 0;
}

/*
 * Full multiply.  transa/transb are 'N' or 'T'.  C_old may be absent
 * (c_nbr < 0) only when beta == 0 and retain == 0.  rows_sel, when not NULL,
 * restricts the computation to the listed (distinct) block rows of the
 * result (the other rows come back empty) -- used to time or check a sample
 * of rows.  Rows are shared among nthreads threads either way.
 * Returns 0 on success, a negative code on bad arguments.
 */
int oracle_multiply(char transa, char transb, double alpha,
                    int32_t a_nbr, int32_t a_nbc, const int32_t *a_rbs, const int32_t *a_cbs,
                    const int64_t *a_rp, const int32_t *a_ci, const double *a_v,
                    int32_t b_nbr, int32_t b_nbc, const int32_t *b_rbs, const int32_t *b_cbs,
                    const int64_t *b_rp, const int32_t *b_ci, const double *b_v,
                    double beta,
                    int32_t c_nbr, int32_t c_nbc, const int32_t *c_rbs, const int32_t *c_cbs,
                    const int64_t *c_rp, const int32_t *c_ci, const double *c_v,
                    double eps, int retain, int nthreads,
                    const int32_t *rows_sel, int64_t n_rows_sel,
                    oracle_result **out) {
  *out = NULL;
  omat A0 = wrap(a_nbr, a_nbc, a_rbs, a_cbs, a_rp, a_ci, a_v);
  omat B0 = wrap(b_nbr, b_nbc, b_rbs, b_cbs, b_rp, b_ci, b_v);
  omat A = (transa == 'T' || transa == 't') ? transpose(&A0) : A0;
  omat B = (transb == 'T' || transb == 't') ? transpose(&B0) : B0;
  int rc = 0;
  omat C0;
  int has_cold = c_nbr >= 0;
  memset(&C0, 0, sizeof(C0));
  if (A.nbc != B.nbr) { rc = -1; goto done; }
  for (int32_t k = 0; k < A.nbc; k++)
    if (A.cbs[k] != B.rbs[k]) { rc = -2; goto done; }
  if ((beta != 0.0 || retain) && !has_cold) { rc = -3; goto done; }
  if (has_cold) {
    C0 = wrap(c_nbr, c_nbc, c_rbs, c_cbs, c_rp, c_ci, c_v);
    if (C0.nbr != A.nbr || C0.nbc != B.nbc) { rc = -4; goto done; }
    for (int32_t i = 0; i < A.nbr; i++) if (C0.rbs[i] != A.rbs[i]) { rc = -5; goto done; }
    for (int32_t j = 0; j < B.nbc; j++) if (C0.cbs[j] != B.cbs[j]) { rc = -5; goto done; }
  }
  {
    double *na = (double *)malloc(sizeof(double) * (size_t)(A.nnzb ? A.nnzb : 1));
    double *nb = (double *)malloc(sizeof(double) * (size_t)(B.nnzb ? B.nnzb : 1));
    all_norms(&A, na);
    all_norms(&B, nb);
    mul_job J;
    J.a = &A; J.b = &B; J.cold = has_cold ? &C0 : NULL;
    J.na = na; J.nb = nb;
    J.alpha = alpha; J.beta = beta; J.eps = eps; J.retain = retain; J.has_cold = has_cold;
    J.rows = (row_out *)calloc((size_t)(A.nbr ? A.nbr : 1), sizeof(row_out));
    pthread_mutex_init(&J.lock, NULL);
    J.sel = NULL;
    J.n_sel = 0;
    if (rows_sel) {
      /* only the selected rows (distinct, in range) */
      for (int64_t s = 0; s < n_rows_sel; s++)
        if (rows_sel[s] < 0 || rows_sel[s] >= A.nbr) { rc = -6; break; }
      char *seen = (char *)calloc((size_t)(A.nbr ? A.nbr : 1), 1);
      for (int64_t s = 0; rc == 0 && s < n_rows_sel; s++) {
        if (seen[rows_sel[s]]) rc = -7;
        seen[rows_sel[s]] = 1;
      }
      free(seen);
      J.sel = rows_sel;
      J.n_sel = n_rows_sel;
    }
    if (rc == 0) {
      J.next = 0;
      int nt = nthreads > 0 ? nthreads : 1;
      pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
      for (int t = 0; t < nt; t++) pthread_create(&th[t], NULL, worker, &J);
      for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
      free(th);
    }
    pthread_mutex_destroy(&J.lock);
    if (rc != 0) {
      free(J.rows); free(na); free(nb);
      goto done;
    }
    /* assemble block CSR */
    oracle_result *R = (oracle_result *)calloc(1, sizeof(oracle_result));
    R->nbr = A.nbr; R->nbc = B.nbc;
    R->rbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A.nbr ? A.nbr : 1));
    R->cbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(B.nbc ? B.nbc : 1));
    memcpy(R->rbs, A.rbs, sizeof(int32_t) * (size_t)A.nbr);
    memcpy(R->cbs, B.cbs, sizeof(int32_t) * (size_t)B.nbc);
    R->row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)A.nbr + 1));
    int64_t tot = 0, totv = 0;
    R->row_ptr[0] = 0;
    for (int32_t i = 0; i < A.nbr; i++) {
      tot += J.rows[i].nb; totv += J.rows[i].nval;
      R->row_ptr[i + 1] = tot;
      R->n_products += J.rows[i].n_products;
      R->n_candidates += J.rows[i].n_candidates;
      R->useful_flops += J.rows[i].flops;
    }
    R->nnzb = tot; R->n_val = totv;
    R->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    R->val = (double *)malloc(sizeof(double) * (size_t)(totv ? totv : 1));
    int64_t pb = 0, pv = 0;
    for (int32_t i = 0; i < A.nbr; i++) {
      row_out *ro = &J.rows[i];
      if (ro->nb) memcpy(R->col_idx + pb, ro->cols, sizeof(int32_t) * (size_t)ro->nb);
      if (ro->nval) memcpy(R->val + pv, ro->val, sizeof(double) * (size_t)ro->nval);
      pb += ro->nb; pv += ro->nval;
      free(ro->cols); free(ro->val);
    }
    free(J.rows); free(na); free(nb);
    *out = R;
  }
done:
  if (has_cold) free(C0.off);
  if (A.own) omat_free(&A);
  if (B.own) omat_free(&B);
  free(A0.off); free(B0.off);
  return rc;
}

/* Post-multiply filter on its own: keep blocks with norm >= eps (R2). */
int oracle_filter(int32_t nbr, int32_t nbc, const int32_t *rbs, const int32_t *cbs,
                  const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                  double eps, oracle_result **out) {
  omat x = wrap(nbr, nbc, rbs, cbs, row_ptr, col_idx, val);
  oracle_result *R = (oracle_result *)calloc(1, sizeof(oracle_result));
  R->nbr = nbr; R->nbc = nbc;
  R->rbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nbr ? nbr : 1));
  R->cbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nbc ? nbc : 1));
  memcpy(R->rbs, rbs, sizeof(int32_t) * (size_t)nbr);
  memcpy(R->cbs, cbs, sizeof(int32_t) * (size_t)nbc);
  R->row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nbr + 1));
  R->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(x.nnzb ? x.nnzb : 1));
  R->val = (double *)malloc(sizeof(double) * (size_t)(x.off[x.nnzb] ? x.off[x.nnzb] : 1));
  int64_t nb = 0, o = 0;
  R->row_ptr[0] = 0;
  for (int32_t i = 0; i < nbr; i++) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      int64_t len = x.off[p + 1] - x.off[p];
      if (block_norm(val + x.off[p], len) < eps) continue;
      R->col_idx[nb++] = col_idx[p];
      memcpy(R->val + o, val + x.off[p], sizeof(double) * (size_t)len);
      o += len;
    }
    R->row_ptr[i + 1] = nb;
  }
  R->nnzb = nb; R->n_val = o;
  free(x.off);
  *out = R;
  return 0;
}

void oracle_free(oracle_result *r) {
  if (!r) return;
  free(r->rbs); free(r->cbs); free(r->row_ptr); free(r->col_idx); free(r->val);
  free(r);
}
