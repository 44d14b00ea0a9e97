// kb_adjoint.hpp -- adjoint of the construction: gradients of L = sum W_ij K_ij.
//
// Not part of the paper; derived from Eq. 7-9.  Per element, with S the symmetric
// nen x nen matrix S_aa = W(E_a, E_a), S_ab = S_ba = W(pair a, b) / 2 (so the element's
// share of L is S : k_e), A = adj(J), G = A dN (so B = G / |J|) and P = G S G^T at
// each integration point (weight w):
//   dL/dc_e  = sum_q w tr(P) / |J|                        (k_e is linear in c),
//   dL/dX_a += c sum_q w / |J|^2 (tr(P) G_a - 2 P G_a)    (G_a = column a of G),
// the second from d|J| = |J| tr(J^{-1} dJ), d(J^{-1}) = -J^{-1} dJ J^{-1}, dJ = dN dX;
// it is c w |J| B^T (tr(M) I - 2 M) with M = B S B^T, written in terms of G.
// All arithmetic is FP64.
//
// Node gradients are sums over the elements at each node.  They are accumulated as the
// same exact fixed-point integers as the assembly (scale from the largest exponent of
// all element contributions; two 64-bit integer chunks per value, summed in LDS per
// workgroup and then globally), so the result does not depend on the order of the
// atomics: bitwise deterministic, exact while a node belongs to at most 2^16 elements.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kb_assemble.hpp"
#include "kb_element.hpp"
#include "kb_kernels.hpp"
#include "kbuild.h"

namespace kb {

// position of (row, col) in a lower CSR with ascending columns, or -1.  The search is
// confined to [0, nnz), the length of col_idx: a row range outside it (a row pointer
// that does not belong to this col_idx) also gives -1.
__device__ __forceinline__ int64_t csr_position(const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col_idx, int64_t nnz, int32_t row,
                                                int32_t col) {
  int64_t lo = row_ptr[row], hi = (int64_t)row_ptr[row + 1] - 1;
  if (lo < 0 || hi >= nnz || lo > hi + 1) return -1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t c = col_idx[mid];
    if (c == col) return mid;
    if (c < col)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// one integration point: P = G S G^T from G (3 x NEN) and the lower triangle of S;
// adds w tr(P) / det to *gc and c w / det^2 (tr(P) G_a - 2 P G_a) to D[a]
template <int NEN>
__device__ __forceinline__ void adjoint_point(const double (&G)[3][NEN], const double (&S)[ElemTraits<NEN>::T],
                                              double det, double w, double c, double* gc, double (&D)[NEN][3]) {
  // T = S G^T (NEN x 3), then P = G T (3 x 3)
  double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
      const double s = a >= b ? S[lidx(a, b)] : S[lidx(b, a)];
      t0 += s * G[0][b];
      t1 += s * G[1][b];
      t2 += s * G[2][b];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      P[i][0] += G[i][a] * t0;
      P[i][1] += G[i][a] * t1;
      P[i][2] += G[i][a] * t2;
    }
  }
  const double tr = P[0][0] + P[1][1] + P[2][2];
  const double inv = 1.0 / det;
  *gc += w * tr * inv;
  const double f = c * w * inv * inv;
#pragma unroll
  for (int a = 0; a < NEN; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      D[a][i] += f * (tr * G[i][a] - 2.0 * (P[i][0] * G[0][a] + P[i][1] * G[1][a] + P[i][2] * G[2][a]));
}

// Per element (one per lane): dL/dc_e into grad_coef, the nen x 3 coordinate
// gradients into gel (element-major), the largest exponent of those into *emax.
template <int NEN>
__global__ __launch_bounds__(128) void k_adjoint_elems(const int32_t* __restrict__ conn,
                                                       const double* __restrict__ coords,
                                                       const double* __restrict__ coef, int64_t n_elem,
                                                       int64_t n_node, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx, int64_t nnz,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ grad_coef, double* __restrict__ gel,
                                                       uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  constexpr int T = ElemTraits<NEN>::T;
  __shared__ uint32_t s_emax;
  if (threadIdx.x == 0) s_emax = 0;
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint32_t em = 0;
  if (e < n_elem) {
    int32_t E[NEN];
    load_conn<NEN>(conn, e, E);
    uint32_t f = check_conn<NEN>(E, n_node);
    double D[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) D[a][0] = D[a][1] = D[a][2] = 0.0;
    double gc = 0.0;
    if (!f) {
      // S from the weights of the element's pairs (off-diagonal pairs at half weight)
      double S[T];
#pragma unroll
      for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          const int32_t row = E[a] > E[b] ? E[a] : E[b], col = E[a] > E[b] ? E[b] : E[a];
          const int64_t k = csr_position(row_ptr, col_idx, nnz, row, col);
          if (k < 0) f |= KB_F_INDEX;
          const double v = k < 0 ? 0.0 : w[k];
          S[lidx(a, b)] = a == b ? v : 0.5 * v;
        }
      double X[NEN][3];
      double X0[3] = {coords[(int64_t)E[0] * 3], coords[(int64_t)E[0] * 3 + 1], coords[(int64_t)E[0] * 3 + 2]};
#pragma unroll
      for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) X[a][j] = a ? coords[(int64_t)E[a] * 3 + j] - X0[j] : 0.0;
      const double c = coef[e];
      if constexpr (NEN == 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double J[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              double s = 0.0;
#pragma unroll
              for (int a = 1; a < 8; ++a) s += hex_dN(q, i, a) * X[a][j];
              J[i][j] = s;
            }
          double A[3][3];
          const double det = adjugate(J, A);
          if (!(det > 0.0)) f |= KB_F_INVERTED;
          double G[3][8];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int a = 0; a < 8; ++a) G[i][a] = A[i][0] * hex_dN(q, 0, a) + A[i][1] * hex_dN(q, 1, a) +
                                                  A[i][2] * hex_dN(q, 2, a);
          adjoint_point<8>(G, S, det, 1.0, c, &gc, D);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        double J[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) J[i][j] = X[i + 1][j];
        double A[3][3];
        const double det = adjugate(J, A);
        if (!(det > 0.0)) f |= KB_F_INVERTED;
        double G[3][4];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          G[i][1] = A[i][0];
          G[i][2] = A[i][1];
          G[i][3] = A[i][2];
          G[i][0] = -(A[i][0] + A[i][1] + A[i][2]);
        }
        adjoint_point<4>(G, S, det, 1.0 / 6.0, c, &gc, D);
      }
    }
    // a degenerate or inverted element, or non-finite input, gives non-finite gradients:
    // flagged, and their node contributions are dropped (the exact sums take 0 for them)
    bool finite = isfinite(gc);
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) finite = finite && isfinite(D[a][j]);
    if (!finite) f |= KB_F_NONFINITE;
    if (f) raise_flag(status, f);
    grad_coef[e] = gc;
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double v = D[a][j];
        gel[(e * NEN + a) * 3 + j] = v;
        const uint32_t ep = (uint32_t)biased_exponent(v);
        em = (ep > em && ep < 0x7FF) ? ep : em;
      }
  }
  if (em) atomicMax(&s_emax, em);
  __syncthreads();
  if (threadIdx.x == 0 && s_emax) atomicMax(emax, s_emax);
}

// Per workgroup, kScatEntries consecutive (element, corner) entries: their coordinate
// gradients are summed per node in an LDS hash table (the same exact chunks, LDS
// atomics), then each distinct node's sums are added once to its global fixed-point
// accumulators acc[node][j] = (low chunk sum, high chunk sum).  Elements numbered with
// locality share most of their nodes within a workgroup, so the global atomics (the
// cost of this step) fall several fold; integer sums keep the result independent of
// the order either way.
constexpr int kScatEntries = 512, kScatSlots = 1024;  // at most half the slots in use

template <int NEN>
__global__ __launch_bounds__(256) void k_adjoint_scatter(const int32_t* __restrict__ conn, int64_t n_elem,
                                                         int64_t n_node, const double* __restrict__ gel,
                                                         const uint32_t* __restrict__ emax,
                                                         unsigned long long* __restrict__ acc) {
  __shared__ int32_t s_node[kScatSlots];
  __shared__ unsigned long long s_acc[kScatSlots][6];
  const int F = 1117 - (int)*emax;
  for (int h = threadIdx.x; h < kScatSlots; h += blockDim.x) {
    s_node[h] = -1;
#pragma unroll
    for (int c = 0; c < 6; ++c) s_acc[h][c] = 0ull;
  }
  __syncthreads();
  const int64_t n = n_elem * NEN;
  const int64_t t0 = (int64_t)blockIdx.x * kScatEntries;
  for (int64_t t = t0 + threadIdx.x; t < t0 + kScatEntries && t < n; t += blockDim.x) {
    const int32_t node = conn[t];
    if (node < 0 || node >= n_node) continue;  // its element was flagged and contributes zeros
    uint32_t h = ((uint32_t)node * 2654435769u) >> (32 - 10);  // kScatSlots = 2^10
    while (true) {  // at most kScatEntries keys in kScatSlots slots: a free slot exists
      const int32_t k = s_node[h];
      if (k == node) break;
      if (k == -1) {
        const int32_t prev = atomicCAS(&s_node[h], -1, node);
        if (prev == -1 || prev == node) break;
      }
      h = (h + 1) & (kScatSlots - 1);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      uint64_t c0;
      int64_t c1;
      to_chunks(gel[t * 3 + j], F, c0, c1);
      if (c0) atomicAdd(&s_acc[h][2 * j], (unsigned long long)c0);
      if (c1) atomicAdd(&s_acc[h][2 * j + 1], (unsigned long long)c1);
    }
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kScatSlots; h += blockDim.x) {
    const int32_t node = s_node[h];
    if (node < 0) continue;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const unsigned long long v = s_acc[h][c];
      if (v) atomicAdd(&acc[(int64_t)node * 6 + c], v);
    }
  }
}

// Per node coordinate: the exact sum converted once (correct rounding) to FP64.
__global__ __launch_bounds__(256) void k_adjoint_nodes(const unsigned long long* __restrict__ acc, int64_t n,
                                                       const uint32_t* __restrict__ emax,
                                                       double* __restrict__ grad_coords) {
  const int F = 1117 - (int)*emax;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t lo, hi;
    join48(acc[2 * i], (int64_t)acc[2 * i + 1], lo, hi);
    grad_coords[i] = from_fixed(lo, hi, F);
  }
}

// zero fill of 64-bit words (a kernel, so the sequence stays capturable in a graph)
__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace kb
