/*
 * kb_oracle.c -- plain FP64 CPU oracle for the lower-triangular global stiffness
 * matrix of the 3D Poisson equation (Ramirez-Gil, Tsuzuki, Montealegre-Rubio,
 * "Global finite element matrix construction based on a CPU-GPU implementation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the HIP library.
 *
 * It follows the paper's definitions directly and makes no attempt at speed:
 *   - Eq. 7-9 (Section 2): k_e = c * sum_q W_q |J_q| B_q^T B_q, with B the 3 x nen
 *     matrix of physical shape-function gradients (the garbled "B = sum grad N_a"
 *     of Eq. 7 is read as the matrix [grad N_1 ... grad N_n]; Section 3 confirms
 *     B = J^{-1} (3x3) times dN (3x8)).
 *   - Section 3 (per-thread pipeline): J = dN (3 x nen) * X (nen x 3), i.e.
 *     J_ij = dx_j / dxi_i; |J| by the 3x3 determinant formula; J^{-1} by the
 *     3x3 inverse formula (adjugate / determinant); B = J^{-1} dN.
 *   - Only the lower triangle (a >= b) of each symmetric k_e is computed
 *     (Section 3, 36 of 64 components for the brick).
 *   - Alg. 1 (serial construction): per element, integrate, map the local pair
 *     (a, b) to a global (row, col), store triplets, then one "sparse" call that
 *     sums duplicates (Eq. 6, K = sum_e k_e) and compresses.  The output here is
 *     lower-triangular CSR: row = max(E_a, E_b), col = min(E_a, E_b); within a row
 *     the columns ascend, so the diagonal comes last.  Entries are structural:
 *     every (row, col) that receives a contribution is stored, even if it sums to 0.
 *
 * Elements: 8-node trilinear brick with the 2x2x2 Gauss-Legendre rule (points
 * +-1/sqrt(3), weights 1; Section 2 and Alg. 2), and the 4-node linear tetrahedron
 * with the one-point centroid rule (weight 1/6), which integrates its constant
 * integrand exactly.  The brick may also be integrated with an n x n x n rule
 * (n = 1..5) for self-checks; the method itself always uses n = 2.
 *
 * Local numbering.  Brick corners in natural coordinates:
 *   0 (-1,-1,-1)  1 (1,-1,-1)  2 (1,1,-1)  3 (-1,1,-1)
 *   4 (-1,-1, 1)  5 (1,-1, 1)  6 (1,1, 1)  7 (-1,1, 1)
 * Tet: N0 = 1 - r - s - t, N1 = r, N2 = s, N3 = t.
 * Lower-triangle storage of one element: position p = a*(a+1)/2 + b for b <= a.
 *
 * Data errors are reported as bit flags (values fixed by the library's ABI):
 *   1 node id out of range, 2 repeated node in one element,
 *   4 non-positive Jacobian determinant at some integration point,
 *   8 non-finite coordinate, coefficient or value.
 * An element with flag 1 or 2 is skipped; the others are integrated as given.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_F_INDEX 1u
#define ORC_F_REPEAT 2u
#define ORC_F_INVERTED 4u
#define ORC_F_NONFINITE 8u

/* ---- Gauss-Legendre points and weights on [-1, 1] (n = 1..5) ---------------- */
/* Classical values (e.g. Zienkiewicz & Taylor, Table of Gauss-Legendre rules). */
int orc_gauss_rule(int n, double* x, double* w) {
  switch (n) {
    case 1:
      x[0] = 0.0; w[0] = 2.0;
      return 0;
    case 2:
      x[0] = -1.0 / sqrt(3.0); x[1] = 1.0 / sqrt(3.0);
      w[0] = 1.0; w[1] = 1.0;
      return 0;
    case 3:
      x[0] = -sqrt(3.0 / 5.0); x[1] = 0.0; x[2] = sqrt(3.0 / 5.0);
      w[0] = 5.0 / 9.0; w[1] = 8.0 / 9.0; w[2] = 5.0 / 9.0;
      return 0;
    case 4: {
      double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
      double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
      double wa = (18.0 + sqrt(30.0)) / 36.0, wb = (18.0 - sqrt(30.0)) / 36.0;
      x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
      w[0] = wb; w[1] = wa; w[2] = wa; w[3] = wb;
      return 0;
    }
    case 5: {
      double a = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
      double b = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
      double wa = (322.0 + 13.0 * sqrt(70.0)) / 900.0, wb = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
      x[0] = -b; x[1] = -a; x[2] = 0.0; x[3] = a; x[4] = b;
      w[0] = wb; w[1] = wa; w[2] = 128.0 / 225.0; w[3] = wa; w[4] = wb;
      return 0;
    }
    default:
      return -1;
  }
}

static const double HEX_NAT[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* dN[i][a] = d N_a / d xi_i of the trilinear brick at natural point (r, s, t). */
static void hex_dN(double r, double s, double t, double dN[3][8]) {
  for (int a = 0; a < 8; ++a) {
    double ra = HEX_NAT[a][0], sa = HEX_NAT[a][1], ta = HEX_NAT[a][2];
    dN[0][a] = ra * (1.0 + sa * s) * (1.0 + ta * t) / 8.0;
    dN[1][a] = (1.0 + ra * r) * sa * (1.0 + ta * t) / 8.0;
    dN[2][a] = (1.0 + ra * r) * (1.0 + sa * s) * ta / 8.0;
  }
}

/* dN of the linear tet (constant). */
static void tet_dN(double dN[3][4]) {
  static const double D[3][4] = {{-1, 1, 0, 0}, {-1, 0, 1, 0}, {-1, 0, 0, 1}};
  memcpy(dN, D, sizeof(D));
}

/*
 * Add one integration point's contribution  W * |J| * B^T B  (lower triangle)
 * into klow.  dN is 3 x nen (row stride 8), X is nen x 3.  Returns |J| (signed).
 */
static double add_point(int nen, const double dN[3][8], const double X[][3], double W, double* klow) {
  double J[3][3];
  /* J = dN * X  (Section 3: dN (3 x nen) times nodal coordinates (nen x 3)) */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int a = 0; a < nen; ++a) s += dN[i][a] * X[a][j];
      J[i][j] = s;
    }
  /* determinant by the 3x3 formula (expansion along the first row) */
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
             - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
             + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  /* inverse by the 3x3 formula: adjugate (transposed cofactors) over det */
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  /* B = J^{-1} dN : column a is the physical gradient of N_a */
  double B[3][8];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < nen; ++a) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += Ji[i][j] * dN[j][a];
      B[i][a] = s;
    }
  /* lower triangle of W |J| B^T B */
  for (int a = 0; a < nen; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += B[i][a] * B[i][b];
      klow[a * (a + 1) / 2 + b] += W * det * s;
    }
  return det;
}

/*
 * Lower triangle of one element matrix (Eq. 9): klow[nen(nen+1)/2].
 * elem = 8 (brick, gauss_n^3 rule) or 4 (tet, centroid rule).  X is nen x 3.
 * Returns flag bits (ORC_F_INVERTED, ORC_F_NONFINITE) or -1 on a bad argument.
 */
int orc_element_lower(int elem, int gauss_n, const double* Xflat, double c, double* klow) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  const double(*X)[3] = (const double(*)[3])Xflat;
  int T = nen * (nen + 1) / 2;
  for (int p = 0; p < T; ++p) klow[p] = 0.0;
  unsigned flags = 0;
  for (int a = 0; a < nen; ++a)
    for (int j = 0; j < 3; ++j)
      if (!isfinite(X[a][j])) flags |= ORC_F_NONFINITE;
  if (!isfinite(c)) flags |= ORC_F_NONFINITE;
  if (elem == 8) {
    double gx[5], gw[5];
    if (orc_gauss_rule(gauss_n, gx, gw) != 0) return -1;
    /* Eq. 9: triple sum over i (r), j (s), k (t) */
    for (int i = 0; i < gauss_n; ++i)
      for (int j = 0; j < gauss_n; ++j)
        for (int k = 0; k < gauss_n; ++k) {
          double dN[3][8];
          hex_dN(gx[i], gx[j], gx[k], dN);
          double det = add_point(8, dN, X, gw[i] * gw[j] * gw[k], klow);
          if (!(det > 0.0)) flags |= ORC_F_INVERTED;
        }
  } else {
    double dN4[3][4], dN[3][8];
    tet_dN(dN4);
    for (int i = 0; i < 3; ++i)
      for (int a = 0; a < 4; ++a) dN[i][a] = dN4[i][a];
    double det = add_point(4, dN, X, 1.0 / 6.0, klow);
    if (!(det > 0.0)) flags |= ORC_F_INVERTED;
  }
  /* c is constant over the element and taken outside the integral (Section 2) */
  for (int p = 0; p < T; ++p) {
    klow[p] *= c;
    if (!isfinite(klow[p])) flags |= ORC_F_NONFINITE;
  }
  return (int)flags;
}

/* Index checks of one element (flag bits ORC_F_INDEX, ORC_F_REPEAT). */
static unsigned check_element(int nen, const int32_t* e, int64_t n_node) {
  unsigned f = 0;
  for (int a = 0; a < nen; ++a)
    if (e[a] < 0 || (int64_t)e[a] >= n_node) f |= ORC_F_INDEX;
  for (int a = 0; a < nen; ++a)
    for (int b = 0; b < a; ++b)
      if (e[a] == e[b]) f |= ORC_F_REPEAT;
  return f;
}

/*
 * Lower values of every element, element-major: out[e * T_e + p].
 * Elements with index errors are left at zero.  Returns the OR of all flags.
 */
int64_t orc_integrate_lower(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                            const double* coords, const double* coef, double* out) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  int T = nen * (nen + 1) / 2;
  unsigned flags = 0;
  double X[8][3];
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    unsigned f = check_element(nen, E, n_node);
    if (f) {
      flags |= f;
      for (int p = 0; p < T; ++p) out[e * T + p] = 0.0;
      continue;
    }
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) X[a][j] = coords[(int64_t)E[a] * 3 + j];
    int r = orc_element_lower(elem, 2, &X[0][0], coef[e], out + e * T);
    if (r < 0) return -1;
    flags |= (unsigned)r;
  }
  return (int64_t)flags;
}

/* ---- assembly: triplets -> sorted, summed lower CSR (Alg. 1 "sparse") ------- */
typedef struct {
  uint64_t key; /* row << 32 | col */
  double val;
} trip_t;

static int cmp_trip(const void* x, const void* y) {
  uint64_t a = ((const trip_t*)x)->key, b = ((const trip_t*)y)->key;
  return (a > b) - (a < b);
}

/*
 * Sort the triplets, sum duplicates and write CSR over the rows [0, n_row).
 * row_ptr[n_row+1]; col_idx / vals have room for cap entries.  Returns nnz;
 * if nnz > cap only row_ptr is written.
 */
static int64_t compress(trip_t* t, int64_t nt, int64_t n_row, int32_t* row_ptr, int32_t* col_idx,
                        double* vals, int64_t cap) {
  qsort(t, (size_t)nt, sizeof(trip_t), cmp_trip);
  int64_t nnz = 0;
  for (int64_t i = 0; i < nt; ++i)
    if (i == 0 || t[i].key != t[i - 1].key) ++nnz;
  for (int64_t r = 0; r <= n_row; ++r) row_ptr[r] = 0;
  int64_t k = -1;
  for (int64_t i = 0; i < nt; ++i) {
    if (i == 0 || t[i].key != t[i - 1].key) {
      ++k;
      int64_t row = (int64_t)(t[i].key >> 32);
      row_ptr[row + 1] += 1;
      if (nnz <= cap) {
        col_idx[k] = (int32_t)(t[i].key & 0xffffffffu);
        vals[k] = 0.0;
      }
    }
    if (nnz <= cap) vals[k] += t[i].val;
  }
  for (int64_t r = 0; r < n_row; ++r) row_ptr[r + 1] += row_ptr[r];
  return nnz;
}

/* Map local pair (a >= b) of element E to its global lower (row, col). */
static uint64_t lower_key(const int32_t* E, int a, int b) {
  uint32_t i = (uint32_t)E[a], j = (uint32_t)E[b];
  uint32_t row = i > j ? i : j, col = i > j ? j : i;
  return ((uint64_t)row << 32) | col;
}

/*
 * Assemble lower CSR K from given element lower values klow[e * T_e + p]
 * (Eq. 6 and Alg. 1 with the integration step supplied by the caller).
 * flags_out receives the index flags.  Returns nnz (>= 0) or -1.
 */
int64_t orc_assemble_lower_csr(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                               const double* klow, int32_t* row_ptr, int32_t* col_idx, double* vals,
                               int64_t cap, uint32_t* flags_out) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  int T = nen * (nen + 1) / 2;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(n_elem * T > 0 ? n_elem * T : 1));
  if (!t) return -1;
  int64_t nt = 0;
  unsigned flags = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    unsigned f = check_element(nen, E, n_node);
    flags |= f;
    if (f) continue;
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b <= a; ++b) {
        t[nt].key = lower_key(E, a, b);
        t[nt].val = klow[e * T + a * (a + 1) / 2 + b];
        ++nt;
      }
  }
  int64_t nnz = compress(t, nt, n_node, row_ptr, col_idx, vals, cap);
  free(t);
  if (flags_out) *flags_out = flags;
  return nnz;
}

/* Full construction (Alg. 1): integrate every element, map, sum, compress. */
int64_t orc_build_lower_csr(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                            const double* coords, const double* coef, int32_t* row_ptr,
                            int32_t* col_idx, double* vals, int64_t cap, uint32_t* flags_out) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  int T = nen * (nen + 1) / 2;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(n_elem * T > 0 ? n_elem * T : 1));
  if (!t) return -1;
  int64_t nt = 0;
  unsigned flags = 0;
  double X[8][3], k[36];
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    unsigned f = check_element(nen, E, n_node);
    flags |= f;
    if (f) continue;
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) X[a][j] = coords[(int64_t)E[a] * 3 + j];
    int r = orc_element_lower(elem, 2, &X[0][0], coef[e], k);
    if (r < 0) {
      free(t);
      return -1;
    }
    flags |= (unsigned)r;
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b <= a; ++b) {
        t[nt].key = lower_key(E, a, b);
        t[nt].val = k[a * (a + 1) / 2 + b];
        ++nt;
      }
  }
  int64_t nnz = compress(t, nt, n_node, row_ptr, col_idx, vals, cap);
  free(t);
  if (flags_out) *flags_out = flags;
  return nnz;
}

/*
 * Entries of selected rows only: for every element touching one of the rows,
 * integrate it and keep the pairs whose global row is selected.  The result is
 * CSR over the selected rows in the order given (rows must be distinct and in
 * range): sel_ptr[n_sel+1], sel_col / sel_val with room for cap entries.
 * Returns the number of entries or -1.
 */
int64_t orc_rows_lower(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                       const double* coords, const double* coef, int64_t n_sel, const int32_t* rows,
                       int32_t* sel_ptr, int32_t* sel_col, double* sel_val, int64_t cap) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  /* slot[node] = position of node in the selection, or -1 */
  int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_node > 0 ? n_node : 1));
  if (!slot) return -1;
  for (int64_t i = 0; i < n_node; ++i) slot[i] = -1;
  for (int64_t s = 0; s < n_sel; ++s) {
    if (rows[s] < 0 || rows[s] >= n_node || slot[rows[s]] != -1) {
      free(slot);
      return -1;
    }
    slot[rows[s]] = (int32_t)s;
  }
  int64_t capt = 1024, nt = 0;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)capt);
  double X[8][3], k[36];
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    if (check_element(nen, E, n_node)) continue;
    int touch = 0;
    for (int a = 0; a < nen; ++a) touch |= slot[E[a]] >= 0;
    if (!touch) continue;
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) X[a][j] = coords[(int64_t)E[a] * 3 + j];
    orc_element_lower(elem, 2, &X[0][0], coef[e], k);
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b <= a; ++b) {
        uint64_t key = lower_key(E, a, b);
        int32_t s = slot[(int64_t)(key >> 32)];
        if (s < 0) continue;
        if (nt == capt) {
          capt *= 2;
          t = (trip_t*)realloc(t, sizeof(trip_t) * (size_t)capt);
        }
        /* re-key by selection position so the CSR follows the given row order */
        t[nt].key = ((uint64_t)(uint32_t)s << 32) | (key & 0xffffffffu);
        t[nt].val = k[a * (a + 1) / 2 + b];
        ++nt;
      }
  }
  int64_t n = compress(t, nt, n_sel, sel_ptr, sel_col, sel_val, cap);
  free(t);
  free(slot);
  return n;
}

/* ---- adjoint of the construction (not in the paper) ---------------------------
 *
 * For a loss L = sum over the lower pattern of W_ij K_ij, W given in the layout of
 * the lower CSR (row_ptr, col_idx) of K, this returns dL/dc (per element) and dL/dX
 * (per node), in FP64.  Derivation from Eq. 7-9:
 *   per element, let S (nen x nen, symmetric) have S_aa = W(E_a, E_a) and
 *   S_ab = S_ba = W(row, col of the pair a, b) / 2 for a != b, so that the element's
 *   share of L is the Frobenius product S : k_e (each off-diagonal global entry takes
 *   k_ab once, and S counts it twice at half weight);
 *   k_e is linear in c, so dL/dc_e = S : k_e / c = sum_q w_q |J_q| tr(B_q S B_q^T);
 *   with M_q = B_q S B_q^T, d|J| = |J| tr(J^{-1} dJ), d(J^{-1}) = -J^{-1} dJ J^{-1} and
 *   dJ = dN dX, one gets dL/dX_e = c sum_q w_q |J_q| B_q^T (tr(M_q) I - 2 M_q), a
 *   nen x 3 block whose row a is added to the gradient of node E_a.
 * Elements with index errors are skipped.  Returns the OR of their flags, or -1 if an
 * element pair has no entry in the given pattern (or on a bad argument).
 */

/* position of (row, col) in the lower CSR, or -1 */
static int64_t csr_find(const int32_t* row_ptr, const int32_t* col_idx, int32_t row, int32_t col) {
  int64_t lo = row_ptr[row], hi = (int64_t)row_ptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (col_idx[mid] == col) return mid;
    if (col_idx[mid] < col)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

/* one integration point of the adjoint: adds w |J| tr(M) to *gc and
 * c w |J| B^T (tr(M) I - 2M) to G (nen x 3) */
static void adjoint_point(int nen, const double dN[3][8], const double X[][3], const double S[8][8], double W,
                          double c, double* gc, double G[8][3]) {
  double J[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int a = 0; a < nen; ++a) s += dN[i][a] * X[a][j];
      J[i][j] = s;
    }
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
             - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
             + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  double B[3][8];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < nen; ++a) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += Ji[i][j] * dN[j][a];
      B[i][a] = s;
    }
  /* M = B S B^T */
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int a = 0; a < nen; ++a)
        for (int b = 0; b < nen; ++b) s += B[i][a] * S[a][b] * B[j][b];
      M[i][j] = s;
    }
  double tr = M[0][0] + M[1][1] + M[2][2];
  *gc += W * det * tr;
  for (int a = 0; a < nen; ++a)
    for (int i = 0; i < 3; ++i) {
      double s = tr * B[i][a];
      for (int j = 0; j < 3; ++j) s -= 2.0 * B[j][a] * M[j][i];
      G[a][i] += c * W * det * s;
    }
}

int64_t orc_adjoint_lower(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn, const double* coords,
                          const double* coef, const int32_t* row_ptr, const int32_t* col_idx, const double* w,
                          double* grad_coef, double* grad_coords) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  for (int64_t i = 0; i < 3 * n_node; ++i) grad_coords[i] = 0.0;
  unsigned flags = 0;
  double gx[5], gw[5];
  orc_gauss_rule(2, gx, gw);
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    grad_coef[e] = 0.0;
    unsigned f = check_element(nen, E, n_node);
    if (f) {
      flags |= f;
      continue;
    }
    double X[8][3], S[8][8], G[8][3];
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) {
        X[a][j] = coords[(int64_t)E[a] * 3 + j];
        G[a][j] = 0.0;
      }
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b < nen; ++b) {
        int32_t row = E[a] > E[b] ? E[a] : E[b], col = E[a] > E[b] ? E[b] : E[a];
        int64_t k = csr_find(row_ptr, col_idx, row, col);
        if (k < 0) return -1;
        S[a][b] = a == b ? w[k] : 0.5 * w[k];
      }
    double gc = 0.0;
    if (elem == 8) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) {
            double dN[3][8];
            hex_dN(gx[i], gx[j], gx[k], dN);
            adjoint_point(8, dN, X, S, gw[i] * gw[j] * gw[k], coef[e], &gc, G);
          }
    } else {
      double dN4[3][4], dN[3][8];
      tet_dN(dN4);
      for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 4; ++a) dN[i][a] = dN4[i][a];
      adjoint_point(4, dN, X, S, 1.0 / 6.0, coef[e], &gc, G);
    }
    grad_coef[e] = gc;
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) grad_coords[(int64_t)E[a] * 3 + j] += G[a][j];
  }
  return (int64_t)flags;
}

/* ---- consistent mass matrix (the closing remark of Section 5) -------------------
 *
 * The same construction with another integrand: m_ab = rho * integral over the element
 * of N_a N_b (rho = the element's coefficient), lower triangle, packed as klow.
 *   Brick: the 2x2x2 Gauss rule of the stiffness matrix, m_ab = rho sum_q |J_q| N_a N_b
 *   at the points (exact for affine bricks: N_a N_b is tri-quadratic in r, s, t).
 *   Tet: the exact integral of the product of two barycentric coordinates,
 *   V (1 + delta_ab) / 20 with V = |J| / 6 (no rule needed).
 * Returns flag bits (ORC_F_INVERTED, ORC_F_NONFINITE) or -1 on a bad argument.
 */
int orc_element_mass_lower(int elem, const double* Xflat, double rho, double* mlow) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  const double(*X)[3] = (const double(*)[3])Xflat;
  int T = nen * (nen + 1) / 2;
  for (int p = 0; p < T; ++p) mlow[p] = 0.0;
  unsigned flags = 0;
  for (int a = 0; a < nen; ++a)
    for (int j = 0; j < 3; ++j)
      if (!isfinite(X[a][j])) flags |= ORC_F_NONFINITE;
  if (!isfinite(rho)) flags |= ORC_F_NONFINITE;
  if (elem == 8) {
    double gx[5], gw[5];
    orc_gauss_rule(2, gx, gw);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
          double r = gx[i], s = gx[j], t = gx[k], dN[3][8], N[8], J[3][3];
          hex_dN(r, s, t, dN);
          for (int a = 0; a < 8; ++a)
            N[a] = (1.0 + HEX_NAT[a][0] * r) * (1.0 + HEX_NAT[a][1] * s) * (1.0 + HEX_NAT[a][2] * t) / 8.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
              double acc = 0.0;
              for (int a = 0; a < 8; ++a) acc += dN[p][a] * X[a][q];
              J[p][q] = acc;
            }
          double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                     - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                     + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
          if (!(det > 0.0)) flags |= ORC_F_INVERTED;
          double W = gw[i] * gw[j] * gw[k];
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b <= a; ++b) mlow[a * (a + 1) / 2 + b] += W * det * N[a] * N[b];
        }
  } else {
    double J[3][3];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) J[p][q] = X[p + 1][q] - X[0][q];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) flags |= ORC_F_INVERTED;
    double V = det / 6.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b <= a; ++b) mlow[a * (a + 1) / 2 + b] = V * (a == b ? 2.0 : 1.0) / 20.0;
  }
  for (int p = 0; p < T; ++p) {
    mlow[p] *= rho;
    if (!isfinite(mlow[p])) flags |= ORC_F_NONFINITE;
  }
  return (int)flags;
}

/* Mass values of every element, element-major (as orc_integrate_lower). */
int64_t orc_integrate_mass_lower(int elem, int64_t n_elem, int64_t n_node, const int32_t* conn,
                                 const double* coords, const double* coef, double* out) {
  int nen = elem;
  if (elem != 8 && elem != 4) return -1;
  int T = nen * (nen + 1) / 2;
  unsigned flags = 0;
  double X[8][3];
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    unsigned f = check_element(nen, E, n_node);
    if (f) {
      flags |= f;
      for (int p = 0; p < T; ++p) out[e * T + p] = 0.0;
      continue;
    }
    for (int a = 0; a < nen; ++a)
      for (int j = 0; j < 3; ++j) X[a][j] = coords[(int64_t)E[a] * 3 + j];
    int r = orc_element_mass_lower(elem, &X[0][0], coef[e], out + e * T);
    if (r < 0) return -1;
    flags |= (unsigned)r;
  }
  return (int64_t)flags;
}

/* ---- several degrees of freedom per node (Alg. 1, Mapping with DOFxn) -------------
 *
 * Element matrices of nen * dof local rows: local DOF p = a * dof + i (node a,
 * component i) is the global DOF dof * E_a + i.  klow[e * T + p(p+1)/2 + q] holds the
 * lower triangle (q <= p) of each element's matrix, T = (nen dof)(nen dof + 1) / 2.
 * The global lower CSR has dof * n_node rows; pairs map to (max, min) of the two global
 * DOFs as in the scalar case.  Returns nnz (>= 0) or -1.
 */
int64_t orc_assemble_lower_csr_dof(int elem, int dof, int64_t n_elem, int64_t n_node, const int32_t* conn,
                                   const double* klow, int32_t* row_ptr, int32_t* col_idx, double* vals,
                                   int64_t cap, uint32_t* flags_out) {
  int nen = elem;
  if ((elem != 8 && elem != 4) || dof < 1 || dof > 3) return -1;
  int nd = nen * dof;
  int64_t T = (int64_t)nd * (nd + 1) / 2;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(n_elem * T > 0 ? n_elem * T : 1));
  if (!t) return -1;
  int64_t nt = 0;
  unsigned flags = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* E = conn + e * nen;
    unsigned f = check_element(nen, E, n_node);
    flags |= f;
    if (f) continue;
    for (int p = 0; p < nd; ++p)
      for (int q = 0; q <= p; ++q) {
        uint32_t gp = (uint32_t)(dof * E[p / dof] + p % dof), gq = (uint32_t)(dof * E[q / dof] + q % dof);
        uint32_t row = gp > gq ? gp : gq, col = gp > gq ? gq : gp;
        t[nt].key = ((uint64_t)row << 32) | col;
        t[nt].val = klow[e * T + (int64_t)p * (p + 1) / 2 + q];
        ++nt;
      }
  }
  int64_t nnz = compress(t, nt, (int64_t)dof * n_node, row_ptr, col_idx, vals, cap);
  free(t);
  if (flags_out) *flags_out = flags;
  return nnz;
}
