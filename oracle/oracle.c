/*
 * oracle.c -- plain, slow, single-threaded reference for general sparse
 * matrix-matrix multiplication C = A*B on CSR inputs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Liu & Vinter, "A Framework for General Sparse
 * Matrix-Matrix Multiplication on GPUs and Heterogeneous Processors"):
 *
 *   - the result of the SpGEMM as defined in Section 2.1: row i of C is the
 *     sum over the stored a_ij of a_ij times row j of B (the row formulation
 *     and Algorithm 1, Gustavson's method), computed with a dense sparse
 *     accumulator ("SPA", the CPU method of Section 2.2).  Every structural
 *     product creates an entry, even if the sums cancel to zero (Section
 *     3.1: the method does not take cancellation into account).  Output
 *     columns are ascending and unique in every row.
 *   - per-row upper bound u_i = sum of nnz(b_j*) over the stored a_ij
 *     (Algorithm 2), the flop count 2*sum(u_i) (Table 2 caption),
 *   - the bin of each row and the size of its row in the temporary matrix
 *     C~ (Algorithm 3, with the paper's fixed thresholds),
 *   - (|A||B|)_ik, the magnitude sum used to scale the value error,
 *   - the gradient of L = <dC, A*B> with respect to the stored values of A
 *     and of B (the product is bilinear, so dA_ij = sum_k dC_ik b_jk and
 *     dB_jk = sum_i a_ij dC_ik over the stored patterns).
 *
 * Arithmetic: IEEE binary64, every product rounded, then added to the
 * running sum in ascending j (ascending position in the row of A), starting
 * from +0.0.  Build with -ffp-contract=off so no fused multiply-add appears.
 * A binary32 variant keeps the accumulator and the products in binary32;
 * it exists only to compare single-precision GPU results bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t m, n, nnz;
  int64_t *row_ptr; /* m+1 */
  int32_t *col;     /* nnz, ascending in each row */
  double *val;      /* nnz, binary64 result (NULL for the binary32 variant) */
  float *val32;     /* nnz, binary32 result (binary32 variant only) */
  double *absval;   /* nnz, (|A||B|)_ik in binary64 */
  int64_t *u;       /* m, Algorithm 2 upper bound per row */
} oracle_result;

void oracle_free(oracle_result *r) {
  if (!r) return;
  free(r->row_ptr);
  free(r->col);
  free(r->val);
  free(r->val32);
  free(r->absval);
  free(r->u);
  free(r);
}

static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

/* Algorithm 2: u_i = sum over stored a_ij of nnz(b_j*).  Returns sum(u_i). */
int64_t oracle_upper_bound(int64_t m, const int64_t *arp, const int32_t *acol,
                           const int64_t *brp, int64_t *u) {
  int64_t total = 0;
  for (int64_t i = 0; i < m; ++i) {
    int64_t ui = 0;
    for (int64_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t j = acol[p];
      ui += brp[j + 1] - brp[j];
    }
    u[i] = ui;
    total += ui;
  }
  return total;
}

/* Algorithm 3 with the paper's thresholds: bins 0 and 1 hold rows of size 0
 * and 1, bins 2..32 one exact size each, bins 33..36 the ranges 33-64,
 * 65-128, 129-256, 257-512, bin 37 everything above 512.  The row of C~ gets
 * u_i entries in bin groups 1-4 and a fixed 256 in group 5.  Returns
 * nnz(C~) = sum of the row sizes. */
int64_t oracle_bin(int64_t m, const int64_t *u, int32_t *bin, int64_t *ctilde) {
  int64_t total = 0;
  for (int64_t i = 0; i < m; ++i) {
    int64_t x = u[i];
    int32_t b;
    int64_t h;
    if (x == 0) {
      b = 0;
      h = 0;
    } else if (x == 1) {
      b = 1;
      h = 1;
    } else if (x >= 2 && x <= 32) {
      b = (int32_t)x;
      h = x;
    } else if (x >= 33 && x <= 64) {
      b = 33;
      h = x;
    } else if (x >= 65 && x <= 128) {
      b = 34;
      h = x;
    } else if (x >= 129 && x <= 256) {
      b = 35;
      h = x;
    } else if (x >= 257 && x <= 512) {
      b = 36;
      h = x;
    } else {
      b = 37;
      h = 256;
    }
    bin[i] = b;
    ctilde[i] = h;
    total += h;
  }
  return total;
}

/* Growable output arrays. */
typedef struct {
  int64_t cap, len;
  int32_t *col;
  double *val;
  float *val32;
  double *absval;
} outbuf;

static int outbuf_reserve(outbuf *o, int64_t need, int want64, int want32) {
  if (need <= o->cap) return 0;
  int64_t cap = o->cap ? o->cap : 1024;
  while (cap < need) cap *= 2;
  int32_t *c = (int32_t *)realloc(o->col, (size_t)cap * sizeof(int32_t));
  if (!c) return -1;
  o->col = c;
  double *a = (double *)realloc(o->absval, (size_t)cap * sizeof(double));
  if (!a) return -1;
  o->absval = a;
  if (want64) {
    double *v = (double *)realloc(o->val, (size_t)cap * sizeof(double));
    if (!v) return -1;
    o->val = v;
  }
  if (want32) {
    float *v = (float *)realloc(o->val32, (size_t)cap * sizeof(float));
    if (!v) return -1;
    o->val32 = v;
  }
  o->cap = cap;
  return 0;
}

/*
 * Gustavson's row-by-row SpGEMM (Algorithm 1) with a dense accumulator.
 * For each row i: for each stored a_ij in ascending j, for each stored b_jk
 * in ascending k, the first product that reaches column k marks it and
 * starts its sum at +0.0; every product is then added to the sum.  The
 * marked columns are sorted and emitted.
 *
 * A: m x k, B: k x n.  Exactly one of (aval64, bval64) / (aval32, bval32)
 * pairs is used: binary64 inputs for the binary64 accumulator, binary32
 * inputs for the binary32 accumulator (acc32 != 0).
 */
static oracle_result *gustavson(int64_t m, int64_t k, int64_t n,
                                const int64_t *arp, const int32_t *acol,
                                const double *aval, const float *aval32,
                                const int64_t *brp, const int32_t *bcol,
                                const double *bval, const float *bval32,
                                int acc32) {
  (void)k;
  oracle_result *r = (oracle_result *)calloc(1, sizeof(oracle_result));
  if (!r) return NULL;
  r->m = m;
  r->n = n;
  r->row_ptr = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
  r->u = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  int64_t *mark = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int32_t *list = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  double *acc = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  float *acc_f = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  double *accabs = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  outbuf o;
  memset(&o, 0, sizeof(o));
  if (!r->row_ptr || !r->u || !mark || !list || !acc || !acc_f || !accabs) goto fail;
  for (int64_t c = 0; c < n; ++c) mark[c] = -1;

  r->row_ptr[0] = 0;
  for (int64_t i = 0; i < m; ++i) {
    int64_t cnt = 0, ui = 0;
    for (int64_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t j = acol[p];
      ui += brp[j + 1] - brp[j];
      for (int64_t q = brp[j]; q < brp[j + 1]; ++q) {
        int32_t c = bcol[q];
        if (mark[c] != i) {
          mark[c] = i;
          list[cnt++] = c;
          acc[c] = 0.0;
          acc_f[c] = 0.0f;
          accabs[c] = 0.0;
        }
        if (acc32) {
          float prod = aval32[p] * bval32[q];
          acc_f[c] = acc_f[c] + prod;
          accabs[c] = accabs[c] + fabs((double)aval32[p]) * fabs((double)bval32[q]);
        } else {
          double prod = aval[p] * bval[q];
          acc[c] = acc[c] + prod;
          accabs[c] = accabs[c] + fabs(aval[p]) * fabs(bval[q]);
        }
      }
    }
    r->u[i] = ui;
    qsort(list, (size_t)cnt, sizeof(int32_t), cmp_i32);
    if (outbuf_reserve(&o, o.len + cnt, !acc32, acc32)) goto fail;
    for (int64_t t = 0; t < cnt; ++t) {
      int32_t c = list[t];
      o.col[o.len] = c;
      if (acc32)
        o.val32[o.len] = acc_f[c];
      else
        o.val[o.len] = acc[c];
      o.absval[o.len] = accabs[c];
      o.len++;
    }
    r->row_ptr[i + 1] = o.len;
  }
  r->nnz = o.len;
  r->col = o.col;
  r->val = o.val;
  r->val32 = o.val32;
  r->absval = o.absval;
  if (!r->col) { /* empty result: hand back valid (tiny) allocations */
    r->col = (int32_t *)malloc(sizeof(int32_t));
    r->absval = (double *)malloc(sizeof(double));
    if (acc32)
      r->val32 = (float *)malloc(sizeof(float));
    else
      r->val = (double *)malloc(sizeof(double));
  }
  free(mark);
  free(list);
  free(acc);
  free(acc_f);
  free(accabs);
  return r;
fail:
  free(mark);
  free(list);
  free(acc);
  free(acc_f);
  free(accabs);
  free(o.col);
  free(o.val);
  free(o.val32);
  free(o.absval);
  r->col = NULL;
  r->val = NULL;
  r->val32 = NULL;
  r->absval = NULL;
  oracle_free(r);
  return NULL;
}

oracle_result *oracle_spgemm_f64(int64_t m, int64_t k, int64_t n,
                                 const int64_t *arp, const int32_t *acol,
                                 const double *aval, const int64_t *brp,
                                 const int32_t *bcol, const double *bval) {
  return gustavson(m, k, n, arp, acol, aval, NULL, brp, bcol, bval, NULL, 0);
}

oracle_result *oracle_spgemm_f32acc(int64_t m, int64_t k, int64_t n,
                                    const int64_t *arp, const int32_t *acol,
                                    const float *aval, const int64_t *brp,
                                    const int32_t *bcol, const float *bval) {
  return gustavson(m, k, n, arp, acol, NULL, aval, brp, bcol, NULL, bval, 1);
}

/* Position of column c in the ascending columns [lo, hi) of a CSR row, or -1. */
static int64_t find_col(const int32_t *col, int64_t lo, int64_t end, int32_t c) {
  int64_t hi = end;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && col[lo] == c) ? lo : -1;
}

/*
 * Gradient of L = sum over S(C) of dC_ik * c_ik, with C = A*B, with respect
 * to the stored values of A and B:
 *   dA_ij = sum over stored b_jk of dC_ik * b_jk          (ascending k)
 *   dB_jk = sum over stored a_ij of a_ij * dC_ik          (ascending i)
 * Every (i,k) reached this way lies in S(C) by construction of C's pattern.
 * If nsa >= 0, only the nsa entries of A listed in sa (positions in A's
 * arrays) are computed (others untouched); likewise nsb / sb for B.  Pass
 * nsa = -1 to compute all of dA, nsa = 0 / dA = NULL to skip it.
 * Returns 0, or -1 if allocation fails, or -2 if a needed (i,k) is missing
 * from C's pattern.
 */
int oracle_grad_f64(int64_t m, int64_t k, int64_t n, const int64_t *arp,
                    const int32_t *acol, const double *aval, const int64_t *brp,
                    const int32_t *bcol, const double *bval, const int64_t *crp,
                    const int32_t *ccol, const double *dc, double *dA,
                    int64_t nsa, const int64_t *sa, double *dB, int64_t nsb,
                    const int64_t *sb) {
  int rc = 0;
  /* row index of every entry of A, for sampled dA */
  int64_t nnzA = arp[m];
  int64_t *arow = NULL, *tptr = NULL, *tpos = NULL;
  if (dA && nsa != 0) {
    arow = (int64_t *)malloc((size_t)(nnzA > 0 ? nnzA : 1) * sizeof(int64_t));
    if (!arow) return -1;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t p = arp[i]; p < arp[i + 1]; ++p) arow[p] = i;
    int64_t cnt = nsa < 0 ? nnzA : nsa;
    for (int64_t t = 0; t < cnt; ++t) {
      int64_t p = nsa < 0 ? t : sa[t];
      int64_t i = arow[p];
      int32_t j = acol[p];
      double s = 0.0;
      for (int64_t q = brp[j]; q < brp[j + 1]; ++q) {
        int64_t pc = find_col(ccol, crp[i], crp[i + 1], bcol[q]);
        if (pc < 0) {
          rc = -2;
          goto done;
        }
        s = s + dc[pc] * bval[q];
      }
      dA[p] = s;
    }
  }
  if (dB && nsb != 0) {
    /* A^T by counting sort: for every column j the entries (i, p) of A with
     * acol[p] == j, in ascending i. */
    tptr = (int64_t *)calloc((size_t)(k + 1), sizeof(int64_t));
    tpos = (int64_t *)malloc((size_t)(nnzA > 0 ? nnzA : 1) * sizeof(int64_t));
    int64_t *trow = (int64_t *)malloc((size_t)(nnzA > 0 ? nnzA : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc((size_t)(k + 1) * sizeof(int64_t));
    int64_t *brow = NULL;
    if (!tptr || !tpos || !trow || !fill) {
      free(trow);
      free(fill);
      rc = -1;
      goto done;
    }
    for (int64_t p = 0; p < nnzA; ++p) tptr[acol[p] + 1]++;
    for (int64_t j = 0; j < k; ++j) tptr[j + 1] += tptr[j];
    memcpy(fill, tptr, (size_t)(k + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i)
      for (int64_t p = arp[i]; p < arp[i + 1]; ++p) {
        int64_t d = fill[acol[p]]++;
        tpos[d] = p;
        trow[d] = i;
      }
    int64_t nnzB = brp[k];
    brow = (int64_t *)malloc((size_t)(nnzB > 0 ? nnzB : 1) * sizeof(int64_t));
    if (!brow) {
      free(trow);
      free(fill);
      rc = -1;
      goto done;
    }
    for (int64_t j = 0; j < k; ++j)
      for (int64_t q = brp[j]; q < brp[j + 1]; ++q) brow[q] = j;
    int64_t cnt = nsb < 0 ? nnzB : nsb;
    for (int64_t t = 0; t < cnt && rc == 0; ++t) {
      int64_t q = nsb < 0 ? t : sb[t];
      int64_t j = brow[q];
      int32_t c = bcol[q];
      double s = 0.0;
      for (int64_t d = tptr[j]; d < tptr[j + 1]; ++d) {
        int64_t i = trow[d];
        int64_t pc = find_col(ccol, crp[i], crp[i + 1], c);
        if (pc < 0) {
          rc = -2;
          break;
        }
        s = s + aval[tpos[d]] * dc[pc];
      }
      dB[q] = s;
    }
    free(brow);
    free(trow);
    free(fill);
  }
done:
  free(arow);
  free(tptr);
  free(tpos);
  return rc;
}
