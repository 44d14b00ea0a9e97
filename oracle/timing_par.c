/*
 * timing_par.c -- all-cores timing harness around the FP64 oracle (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY, like kb_oracle.c, which it is linked with: it exists to time
 * the oracle's construction on every host core, as a CPU reference beside the
 * single-threaded oracle.  The arithmetic is the oracle's own: each element goes through
 * orc_element_lower (Eq. 7-9 with the element's rule), its lower pairs are mapped to
 * (max, min) global indices (Alg. 1), and duplicates are summed into lower CSR (Eq. 6).
 * Only the loop structure differs:
 *   - elements are integrated in parallel (OpenMP), each writing its triplets at a
 *     fixed place (invalid elements leave keys that sort after every real one);
 *   - the triplets are sorted by key with a parallel merge sort (one qsort per thread,
 *     then rounds of pairwise merges, each round's merges in parallel);
 *   - runs of equal keys are summed in parallel over key-aligned chunks.
 * Duplicate keys are summed in sorted order, which may differ from the serial oracle's
 * (qsort is not stable): the values agree to rounding, the pattern exactly.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int orc_element_lower(int elem, int gauss_n, const double* Xflat, double c, double* klow);

typedef struct {
  uint64_t key; /* row << 32 | col */
  double val;
} ptrip_t;

static int cmp_ptrip(const void* x, const void* y) {
  uint64_t a = ((const ptrip_t*)x)->key, b = ((const ptrip_t*)y)->key;
  return (a > b) - (a < b);
}

static void merge_runs(const ptrip_t* a, int64_t na, const ptrip_t* b, int64_t nb, ptrip_t* out) {
  int64_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) out[k++] = (b[j].key < a[i].key) ? b[j++] : a[i++];
  while (i < na) out[k++] = a[i++];
  while (j < nb) out[k++] = b[j++];
}

/* sort t[0..n) with `threads` threads; tmp has room for n triplets; returns the buffer
 * holding the result (t or tmp) */
static ptrip_t* par_sort(ptrip_t* t, ptrip_t* tmp, int64_t n, int threads) {
  int64_t nrun = threads;
  int64_t* bound = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nrun + 1));
  for (int64_t r = 0; r <= nrun; ++r) bound[r] = n * r / nrun;
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t r = 0; r < nrun; ++r) qsort(t + bound[r], (size_t)(bound[r + 1] - bound[r]), sizeof(ptrip_t), cmp_ptrip);
  ptrip_t *src = t, *dst = tmp;
  for (int64_t width = 1; width < nrun; width *= 2) {
#pragma omp parallel for num_threads(threads) schedule(dynamic)
    for (int64_t r = 0; r < nrun; r += 2 * width) {
      const int64_t lo = bound[r], mid = bound[r + width < nrun ? r + width : nrun];
      const int64_t hi = bound[r + 2 * width < nrun ? r + 2 * width : nrun];
      merge_runs(src + lo, mid - lo, src + mid, hi - mid, dst + lo);
    }
    ptrip_t* s = src;
    src = dst;
    dst = s;
  }
  free(bound);
  return src;
}

/*
 * Full construction on `threads` threads (0: all).  Same arguments and results as
 * orc_build_lower_csr: returns nnz (>= 0) or -1; only row_ptr is written if nnz > cap.
 */
int64_t orc_par_build_lower_csr(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                                const double* coords, const double* coef, int32_t* row_ptr, int32_t* col_idx,
                                double* vals, int64_t cap, uint32_t* flags_out, int threads) {
  if (elem != 8 && elem != 4) return -1;
  if (threads <= 0) threads = omp_get_max_threads();
  const int nen = elem, T = nen * (nen + 1) / 2;
  const int64_t nt = n_elem * T;
  ptrip_t* t = (ptrip_t*)malloc(sizeof(ptrip_t) * (size_t)(nt > 0 ? nt : 1));
  ptrip_t* tmp = (ptrip_t*)malloc(sizeof(ptrip_t) * (size_t)(nt > 0 ? nt : 1));
  if (!t || !tmp) {
    free(t);
    free(tmp);
    return -1;
  }
  unsigned flags = 0;
  int bad = 0;
#pragma omp parallel num_threads(threads) reduction(| : flags) reduction(| : bad)
  {
    double X[8][3], k[36];
#pragma omp for schedule(static)
    for (int64_t e = 0; e < n_elem; ++e) {
      const int32_t* E = conn + e * nen;
      unsigned f = 0;
      for (int a = 0; a < nen; ++a)
        if (E[a] < 0 || (int64_t)E[a] >= n_node) f |= 1u; /* index */
      for (int a = 0; a < nen; ++a)
        for (int b = 0; b < a; ++b)
          if (E[a] == E[b]) f |= 2u; /* repeat */
      ptrip_t* out = t + e * T;
      if (f) {
        flags |= f;
        for (int p = 0; p < T; ++p) out[p].key = UINT64_MAX, out[p].val = 0.0;
        continue;
      }
      for (int a = 0; a < nen; ++a)
        for (int j = 0; j < 3; ++j) X[a][j] = coords[(int64_t)E[a] * 3 + j];
      int r = orc_element_lower(elem, 2, &X[0][0], coef[e], k);
      if (r < 0) bad = 1;
      flags |= (unsigned)(r > 0 ? r : 0);
      for (int a = 0; a < nen; ++a)
        for (int b = 0; b <= a; ++b) {
          uint32_t i = (uint32_t)E[a], j = (uint32_t)E[b];
          out->key = ((uint64_t)(i > j ? i : j) << 32) | (i > j ? j : i);
          out->val = k[a * (a + 1) / 2 + b];
          ++out;
        }
    }
  }
  if (bad) {
    free(t);
    free(tmp);
    return -1;
  }
  ptrip_t* s = par_sort(t, tmp, nt, threads);
  int64_t n = nt; /* drop the invalid elements' keys (sorted last) */
  while (n > 0 && s[n - 1].key == UINT64_MAX) --n;
  /* chunks that start at a new key: each thread counts and then writes its entries */
  int64_t* cb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(threads + 1));
  int64_t* cu = (int64_t*)calloc((size_t)threads + 1, sizeof(int64_t));
  for (int c = 0; c <= threads; ++c) {
    int64_t b = n * c / threads;
    while (b > 0 && b < n && s[b].key == s[b - 1].key) ++b;
    cb[c] = b;
  }
  for (int c = 1; c <= threads; ++c)
    if (cb[c] < cb[c - 1]) cb[c] = cb[c - 1];
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int c = 0; c < threads; ++c) {
    int64_t u = 0;
    for (int64_t i = cb[c]; i < cb[c + 1]; ++i)
      if (i == cb[c] || s[i].key != s[i - 1].key) ++u;
    cu[c + 1] = u;
  }
  for (int c = 0; c < threads; ++c) cu[c + 1] += cu[c];
  const int64_t nnz = cu[threads];
  memset(row_ptr, 0, sizeof(int32_t) * (size_t)(n_node + 1));
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int c = 0; c < threads; ++c) {
    int64_t k = cu[c] - 1;
    for (int64_t i = cb[c]; i < cb[c + 1]; ++i) {
      if (i == cb[c] || s[i].key != s[i - 1].key) {
        ++k;
#pragma omp atomic
        row_ptr[(s[i].key >> 32) + 1] += 1;
        if (nnz <= cap) {
          col_idx[k] = (int32_t)(s[i].key & 0xffffffffu);
          vals[k] = 0.0;
        }
      }
      if (nnz <= cap) vals[k] += s[i].val;
    }
  }
  for (int64_t r = 0; r < n_node; ++r) row_ptr[r + 1] += row_ptr[r];
  free(cb);
  free(cu);
  free(t);
  free(tmp);
  if (flags_out) *flags_out = flags;
  return nnz;
}

/* threads the harness uses when asked for 0 (OpenMP's default on this host) */
int orc_par_max_threads(void) { return omp_get_max_threads(); }
