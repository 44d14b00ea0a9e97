// kb_element.hpp -- per-lane element integration for gfx950 (one element per lane).
//
// Lower triangle of k_e = c * sum_q W_q |J_q| B_q^T B_q (Eq. 7-9), computed as in the
// per-thread pipeline of Section 3 / Alg. 2: J = dN X, |J| by the 3x3 determinant
// formula, J^{-1} by the 3x3 adjugate formula, B = J^{-1} dN, lower triangle only.
//
// Arithmetic form used here (same mathematics, fewer operations):
//   A = adj(J) (so J^{-1} = A / |J|),  G = A dN  (so B = G / |J|),
//   W |J| B^T B = (W / |J|) G^T G.
// X holds node coordinates minus those of local node 0 (translation does not change
// J), formed in FP64 before any conversion, so FP32 geometry never suffers the
// cancellation of absolute coordinates.
//
// Shape-function derivatives at the integration points are compile-time constants:
// every loop over points and nodes is fully unrolled, so they become instruction
// literals instead of table loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kb {

// ---- brick: natural corner signs (corner order of the C ABI) ----------------------
__host__ __device__ constexpr int hex_sign(int a, int dir) {
  // dir 0: r, 1: s, 2: t
  return dir == 0 ? ((a == 1 || a == 2 || a == 5 || a == 6) ? 1 : -1)
       : dir == 1 ? ((a == 2 || a == 3 || a == 6 || a == 7) ? 1 : -1)
                  : (a >= 4 ? 1 : -1);
}

// 1/sqrt(3): abscissa of the two-point Gauss-Legendre rule (weights 1).
constexpr double kGauss2 = 0.57735026918962576450914878050195746;

// natural coordinate of integration point q (0..7) along dir: q = 4 i + 2 j + k
__host__ __device__ constexpr double hex_qp(int q, int dir) {
  return ((dir == 0 ? (q >> 2) : dir == 1 ? (q >> 1) : q) & 1) ? kGauss2 : -kGauss2;
}

// dN_a / d xi_dir of the trilinear brick at point q:
//   d/dr N_a = r_a (1 + s_a s)(1 + t_a t) / 8, and cyclically.
__host__ __device__ constexpr double hex_dN(int q, int dir, int a) {
  const double r = hex_qp(q, 0), s = hex_qp(q, 1), t = hex_qp(q, 2);
  const double ra = hex_sign(a, 0), sa = hex_sign(a, 1), ta = hex_sign(a, 2);
  return dir == 0 ? ra * (1.0 + sa * s) * (1.0 + ta * t) / 8.0
       : dir == 1 ? (1.0 + ra * r) * sa * (1.0 + ta * t) / 8.0
                  : (1.0 + ra * r) * (1.0 + sa * s) * ta / 8.0;
}

__host__ __device__ constexpr int lidx(int a, int b) { return a * (a + 1) / 2 + b; }

template <typename T>
__device__ __forceinline__ T kabs(T x) {
  return x < T(0) ? -x : x;
}

// adjugate A of J (J^{-1} = A / det) and det J
template <typename T>
__device__ __forceinline__ T adjugate(const T (&J)[3][3], T (&A)[3][3]) {
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
}

// Estimated infinity-norm condition number ||J|| ||J^{-1}|| = ||J|| ||A|| / |det|,
// tested without division: returns true if ||J|| ||A|| > tau |det| (or det is not finite/positive).
template <typename T>
__device__ __forceinline__ bool ill_conditioned(const T (&J)[3][3], const T (&A)[3][3], T det, T tau) {
  T nj = T(0), na = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T sj = kabs(J[i][0]) + kabs(J[i][1]) + kabs(J[i][2]);
    T sa = kabs(A[i][0]) + kabs(A[i][1]) + kabs(A[i][2]);
    nj = sj > nj ? sj : nj;
    na = sa > na ? sa : na;
  }
  return !(nj * na <= tau * det);
}

// ---- brick, one precision for geometry (GT) and one for G / accumulation (AT) -------
// X[a][j] = x_j(node a) - x_j(node 0) for a = 1..7.  k[36] += lower of the element
// integral (without c).  Returns false if some det is not > 0.  If CHECK, *need_fb
// is set when a point's Jacobian is ill-conditioned (estimate > tau).
template <typename GT, typename AT, bool CHECK>
__device__ __forceinline__ bool hex_integrate(const GT (&X)[8][3], AT (&k)[36], GT tau, bool* need_fb) {
  bool ok = true;
#pragma unroll
  for (int p = 0; p < 36; ++p) k[p] = AT(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    GT J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GT s = GT(0);
#pragma unroll
        for (int a = 1; a < 8; ++a) s += GT(hex_dN(q, i, a)) * X[a][j];
        J[i][j] = s;
      }
    GT A[3][3];
    const GT det = adjugate(J, A);
    ok = ok && (det > GT(0));
    if (CHECK) {
      if (ill_conditioned(J, A, det, tau)) *need_fb = true;
    }
    // G = A dN (3 x 8), accumulated in AT
    AT G[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        AT s = AT(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) s += AT(A[i][j]) * AT(hex_dN(q, j, a));
        G[i][a] = s;
      }
    // weight W = 1 for every point of the 2x2x2 rule
    const AT f = AT(GT(1) / det);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const AT g0 = f * G[0][a], g1 = f * G[1][a], g2 = f * G[2][a];
#pragma unroll
      for (int b = 0; b <= a; ++b) k[lidx(a, b)] += g0 * G[0][b] + g1 * G[1][b] + g2 * G[2][b];
    }
    // keep the eight points in sequence: interleaving them only raises register pressure
    __builtin_amdgcn_sched_barrier(0);
  }
  return ok;
}

// Half of the 2x2x2 rule, for two lanes sharing one brick: the four points with r = -g
// (h = 0) or r = +g (h = 1).  The same arithmetic per point as hex_integrate; the
// derivatives of the lane's half are picked once per point from the two constants.
template <typename GT, typename AT, bool CHECK>
__device__ __forceinline__ bool hex_integrate_half(const GT (&X)[8][3], AT (&k)[36], GT tau, bool* need_fb, int h) {
  bool ok = true;
#pragma unroll
  for (int p = 0; p < 36; ++p) k[p] = AT(0);
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    GT dN[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int a = 0; a < 8; ++a) dN[i][a] = h ? GT(hex_dN(4 + qq, i, a)) : GT(hex_dN(qq, i, a));
    GT J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GT s = GT(0);
#pragma unroll
        for (int a = 1; a < 8; ++a) s += dN[i][a] * X[a][j];
        J[i][j] = s;
      }
    GT A[3][3];
    const GT det = adjugate(J, A);
    ok = ok && (det > GT(0));
    if (CHECK) {
      if (ill_conditioned(J, A, det, tau)) *need_fb = true;
    }
    AT G[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        AT s = AT(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) s += AT(A[i][j]) * AT(dN[j][a]);
        G[i][a] = s;
      }
    const AT f = AT(GT(1) / det);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const AT g0 = f * G[0][a], g1 = f * G[1][a], g2 = f * G[2][a];
#pragma unroll
      for (int b = 0; b <= a; ++b) k[lidx(a, b)] += g0 * G[0][b] + g1 * G[1][b] + g2 * G[2][b];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return ok;
}

// ---- tetrahedron: J rows are the edge vectors from node 0 (dN constant) -------------
// X[a][j] = x_j(node a) - x_j(node 0), a = 1..3.  One point, weight 1/6.
template <typename GT, typename AT, bool CHECK>
__device__ __forceinline__ bool tet_integrate(const GT (&X)[4][3], AT (&k)[10], GT tau, bool* need_fb) {
  GT J[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) J[i][j] = X[i + 1][j];
  GT A[3][3];
  const GT det = adjugate(J, A);
  if (CHECK) {
    if (ill_conditioned(J, A, det, tau)) *need_fb = true;
  }
  // G = A dN with dN = [[-1,1,0,0],[-1,0,1,0],[-1,0,0,1]]: column a >= 1 is A[:, a-1]
  AT G[3][4];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    G[i][1] = AT(A[i][0]);
    G[i][2] = AT(A[i][1]);
    G[i][3] = AT(A[i][2]);
    G[i][0] = -(G[i][1] + G[i][2] + G[i][3]);
  }
  const AT f = AT(GT(1) / (GT(6) * det));
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const AT g0 = f * G[0][a], g1 = f * G[1][a], g2 = f * G[2][a];
#pragma unroll
    for (int b = 0; b <= a; ++b) k[lidx(a, b)] = g0 * G[0][b] + g1 * G[1][b] + g2 * G[2][b];
  }
  return det > GT(0);
}

// ---- consistent mass matrix: m_ab = integral of N_a N_b (c applied by the caller) ------
// N_a at brick point q: (1 + r_a r)(1 + s_a s)(1 + t_a t) / 8
__host__ __device__ constexpr double hex_N(int q, int a) {
  return (1.0 + hex_sign(a, 0) * hex_qp(q, 0)) * (1.0 + hex_sign(a, 1) * hex_qp(q, 1)) *
         (1.0 + hex_sign(a, 2) * hex_qp(q, 2)) / 8.0;
}

// brick: sum over the 2x2x2 points of |J_q| N_a N_b (exact for affine bricks)
template <typename GT, typename AT, bool CHECK>
__device__ __forceinline__ bool hex_mass(const GT (&X)[8][3], AT (&m)[36], GT tau, bool* need_fb) {
  bool ok = true;
#pragma unroll
  for (int p = 0; p < 36; ++p) m[p] = AT(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    GT J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GT s = GT(0);
#pragma unroll
        for (int a = 1; a < 8; ++a) s += GT(hex_dN(q, i, a)) * X[a][j];
        J[i][j] = s;
      }
    GT A[3][3];
    const GT det = adjugate(J, A);
    ok = ok && (det > GT(0));
    if (CHECK) {
      if (ill_conditioned(J, A, det, tau)) *need_fb = true;
    }
    const AT d = AT(det);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) m[lidx(a, b)] += d * AT(hex_N(q, a) * hex_N(q, b));
    __builtin_amdgcn_sched_barrier(0);
  }
  return ok;
}

// tetrahedron: the exact integral of two barycentric coordinates, V (1 + delta_ab) / 20
// with V = |J| / 6
template <typename GT, typename AT, bool CHECK>
__device__ __forceinline__ bool tet_mass(const GT (&X)[4][3], AT (&m)[10], GT tau, bool* need_fb) {
  GT J[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) J[i][j] = X[i + 1][j];
  GT A[3][3];
  const GT det = adjugate(J, A);
  if (CHECK) {
    if (ill_conditioned(J, A, det, tau)) *need_fb = true;
  }
  const AT f = AT(det) / AT(120);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) m[lidx(a, b)] = a == b ? AT(2) * f : f;
  return det > GT(0);
}

// packed lower-triangle entries of an element matrix of NEN rows (NEN = nodes times
// degrees of freedom per node)
template <int NEN>
struct ElemTraits {
  static constexpr int T = NEN * (NEN + 1) / 2;
};

// the element integrand: stiffness (Eq. 7-9) or consistent mass
enum class Op { Stiffness = 0, Mass = 1 };

template <int NEN, typename GT, typename AT, bool CHECK, Op OP = Op::Stiffness>
__device__ __forceinline__ bool integrate(const GT (&X)[NEN][3], AT (&k)[ElemTraits<NEN>::T], GT tau, bool* need_fb) {
  if constexpr (OP == Op::Mass) {
    if constexpr (NEN == 8)
      return hex_mass<GT, AT, CHECK>(X, k, tau, need_fb);
    else
      return tet_mass<GT, AT, CHECK>(X, k, tau, need_fb);
  } else {
    if constexpr (NEN == 8)
      return hex_integrate<GT, AT, CHECK>(X, k, tau, need_fb);
    else
      return tet_integrate<GT, AT, CHECK>(X, k, tau, need_fb);
  }
}

}  // namespace kb
