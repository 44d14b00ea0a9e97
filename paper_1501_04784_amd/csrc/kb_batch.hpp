// kb_batch.hpp -- many independent meshes built as one block-diagonal matrix.
//
// A batch packs its meshes back to back (elements [elem_off[m], elem_off[m+1]), nodes
// [node_off[m], node_off[m+1]), connectivity in mesh-local node ids).  Shifting each
// mesh's ids by node_off[m] gives one mesh whose K is block diagonal (no element spans
// two meshes), so one pass of the ordinary pipeline builds every mesh's matrix at once;
// its CSR lists the meshes' rows in order.  Each mesh's own CSR is then that block with
// its row pointers rebased to 0 and its columns shifted back to local ids.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kb_kernels.hpp"
#include "kbuild.h"

namespace kb {

// largest m in [0, n) with off[m] <= i (off non-decreasing, off[0] <= i)
__device__ __forceinline__ int64_t owner_of(const int64_t* __restrict__ off, int64_t n, int64_t i) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One thread per mesh (and one more): offsets must start at 0, not decrease and end at
// the totals; any violation sets KB_F_INDEX in *flags (no element is then trusted to
// belong to the mesh it claims, and the shifted ids are checked again by the pipeline).
__global__ void k_batch_check(const int64_t* __restrict__ elem_off, const int64_t* __restrict__ node_off,
                              int64_t n_mesh, int64_t n_elem, int64_t n_node, uint32_t* __restrict__ flags) {
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (m > n_mesh) return;
  bool bad = false;
  if (m == 0) bad = elem_off[0] != 0 || node_off[0] != 0;
  if (m == n_mesh) bad = bad || elem_off[n_mesh] != n_elem || node_off[n_mesh] != n_node;
  if (m < n_mesh) bad = bad || elem_off[m + 1] < elem_off[m] || node_off[m + 1] < node_off[m];
  if (bad) atomicOr(flags, KB_F_INDEX);
}

// Global connectivity: each element's local ids shifted by its mesh's first node.  A
// local id outside [0, nodes of the mesh) becomes -1, which the pipeline flags as an
// index error and leaves out.  When the offsets failed their check (*flags set) no
// element can be placed in a mesh: every id becomes -1.
template <int NEN>
__global__ __launch_bounds__(256) void k_batch_conn(const int32_t* __restrict__ conn, const int64_t* __restrict__ elem_off,
                                                    const int64_t* __restrict__ node_off, int64_t n_mesh,
                                                    int64_t n_elem, const uint32_t* __restrict__ flags,
                                                    int32_t* __restrict__ gconn) {
  const bool bad = *flags != 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elem;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (bad) {
#pragma unroll
      for (int a = 0; a < NEN; ++a) gconn[e * NEN + a] = -1;
      continue;
    }
    const int64_t m = owner_of(elem_off, n_mesh, e);
    const int64_t base = node_off[m], nm = node_off[m + 1] - base;
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
      const int32_t v = conn[e * NEN + a];
      gconn[e * NEN + a] = (v >= 0 && v < nm) ? (int32_t)(base + v) : -1;
    }
  }
}

// One thread per node i of the batch (mesh m): its row in mesh m's own CSR.  row_ptr of
// mesh m occupies out_ptr[node_off[m] + m .. node_off[m+1] + m]; columns become local.
// Columns are rewritten only when the union CSR was written (nnz <= cap).  Offsets that
// failed their check (*flags set) say nothing trustworthy about where a mesh's rows
// go: then every one of the n_node + n_mesh row pointers is written as 0 instead (no
// element was kept, so the union CSR is empty) and node_off is not read.
__global__ __launch_bounds__(256) void k_batch_rows(const int32_t* __restrict__ uptr, const int64_t* __restrict__ node_off,
                                                    int64_t n_mesh, int64_t n_node, int64_t cap,
                                                    const uint32_t* __restrict__ flags,
                                                    int32_t* __restrict__ col_idx, int32_t* __restrict__ out_ptr) {
  if (*flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_node + n_mesh;
         i += (int64_t)gridDim.x * blockDim.x)
      out_ptr[i] = 0;
    return;
  }
  const int64_t nnz = uptr[n_node];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_node;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = owner_of(node_off, n_mesh, i);
    const int64_t base = node_off[m];
    out_ptr[i + m] = uptr[i] - uptr[base];
    if (nnz <= cap)
      for (int32_t k = uptr[i]; k < uptr[i + 1]; ++k) col_idx[k] -= (int32_t)base;
  }
}

// One thread per mesh: its closing row pointer and its first entry in col_idx / vals;
// nnz_off[n_mesh] already holds the batch total.  Folds the offset-check flags into the
// status word.  With failed offsets (*flags set) node_off is not read: every mesh gets
// the empty range nnz_off[m] = 0 (k_batch_rows has zeroed the row pointers).
__global__ void k_batch_meshes(const int32_t* __restrict__ uptr, const int64_t* __restrict__ node_off,
                               int64_t n_mesh, const uint32_t* __restrict__ flags, int32_t* __restrict__ out_ptr,
                               int64_t* __restrict__ nnz_off, uint32_t* __restrict__ status) {
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const uint32_t bad = *flags;
  if (m == 0 && bad) atomicOr(status, bad);
  if (m >= n_mesh) return;
  if (bad) {
    nnz_off[m] = 0;
    return;
  }
  const int64_t b = node_off[m], e = node_off[m + 1];
  out_ptr[e + m] = uptr[e] - uptr[b];
  nnz_off[m] = uptr[b];
}

}  // namespace kb
