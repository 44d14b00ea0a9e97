// kb_kernels.hpp -- gfx950 kernels of the lower-triangular stiffness build.
//
// Shared pieces: connectivity checks, node ranks, device-wide int32 scan, the
// per-element integration wrapper (precision modes, FP64 fallback, flags) and the
// element-major integration kernel.  The assembly kernels are in kb_assemble.hpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kb_element.hpp"
#include "kbuild.h"

namespace kb {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ __forceinline__ void raise_flag(uint32_t* status, uint32_t f) { atomicOr(status, f); }

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8).
// Map b to a work item so that each XCD takes one contiguous range of the n items: the
// runs that neighbouring items write next to each other then meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t n) {
  const int64_t x = b % kXcds, i = b / kXcds, full = n / kXcds, rem = n % kXcds;
  return x * full + (x < rem ? x : rem) + i;
}

template <int NEN>
__device__ __forceinline__ void load_conn(const int32_t* __restrict__ conn, int64_t e, int32_t (&E)[NEN]) {
#pragma unroll
  for (int a = 0; a < NEN; ++a) E[a] = conn[e * NEN + a];
}

// KB_F_INDEX / KB_F_REPEAT bits of one element
template <int NEN>
__device__ __forceinline__ uint32_t check_conn(const int32_t (&E)[NEN], int64_t n_node) {
  uint32_t f = 0;
#pragma unroll
  for (int a = 0; a < NEN; ++a)
    if (E[a] < 0 || (int64_t)E[a] >= n_node) f |= KB_F_INDEX;
#pragma unroll
  for (int a = 0; a < NEN; ++a)
#pragma unroll
    for (int b = 0; b < a; ++b)
      if (E[a] == E[b]) f |= KB_F_REPEAT;
  return f;
}

// rank of each node among the element's (distinct) ids
template <int NEN>
__device__ __forceinline__ void node_ranks(const int32_t (&E)[NEN], int (&r)[NEN]) {
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    int s = 0;
#pragma unroll
    for (int b = 0; b < NEN; ++b) s += (E[b] < E[a]) ? 1 : 0;
    r[a] = s;
  }
}

// ---------------------------------------------------------------- several DOFs
// Connectivity of the DOF view of a mesh with dof components per node: entry a*dof+i
// of element e is the global DOF dof*E[a]+i.  An id outside [0, n_node) maps to ids
// outside [0, dof*n_node) (a negative one stays negative; distinct ids stay distinct
// below 2^31/dof in magnitude), so the pipeline flags the element as the node ids would.
__global__ __launch_bounds__(256) void k_dof_conn(const int32_t* __restrict__ conn, int64_t n, int dof,
                                                  int32_t* __restrict__ dconn) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = conn[t];
    for (int i = 0; i < dof; ++i) {
      int64_t w = dof * v + i;
      w = w > INT32_MAX ? INT32_MAX : (w < INT32_MIN ? INT32_MIN : w);
      dconn[t * dof + i] = (int32_t)w;
    }
  }
}

// ------------------------------------------------------------------------- fill
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_init_status(uint32_t* __restrict__ status, int64_t* __restrict__ nnz) {
  if (threadIdx.x < KB_STATUS_WORDS) status[threadIdx.x] = 0u;
  if (threadIdx.x == 0 && nnz) *nnz = 0;
}

// --------------------------------------------------------------------- scan (int32)
// block-wide exclusive scan of one value per thread; returns the block total in *total
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* smem_waves, int32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) smem_waves[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < nwaves; ++w) {
      int32_t t = smem_waves[w];
      smem_waves[w] = s;
      s += t;
    }
    smem_waves[nwaves] = s;
  }
  __syncthreads();
  const int32_t r = x - v + smem_waves[wave];
  *total = smem_waves[nwaves];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(const int32_t* __restrict__ in, int64_t n,
                                                                int32_t* __restrict__ partials) {
  __shared__ int32_t sw[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  int32_t total;
  block_exclusive_scan(s, sw, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// single block: exclusive scan of partials[0..nb) in place
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t* __restrict__ partials, int64_t nb) {
  __shared__ int32_t sw[kScanThreads / 64 + 1];
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += (int64_t)kScanThreads * kScanItems) {
    const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (my + i < nb) ? partials[my + i] : 0;
      s += v[i];
    }
    int32_t total;
    int32_t off = block_exclusive_scan(s, sw, &total) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (my + i < nb) partials[my + i] = off;
      off += v[i];
    }
    carry += total;
  }
}

// out[0..n] = exclusive scan of in[0..n) (out[n] = total); total64 optional
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t* __restrict__ in, int64_t n,
                                                            const int32_t* __restrict__ partials,
                                                            int32_t* __restrict__ out, int64_t* __restrict__ total64) {
  __shared__ int32_t sw[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int32_t total;
  int32_t off = block_exclusive_scan(s, sw, &total) + partials[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = off;
    off += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const int32_t grand = partials[blockIdx.x] + total;
    out[n] = grand;
    if (total64) *total64 = grand;
  }
}

// n == 0: out[0] = 0
__global__ void k_scan_empty(int32_t* __restrict__ out, int64_t* __restrict__ total64) {
  out[0] = 0;
  if (total64) *total64 = 0;
}

// --------------------------------------------------------------------- integrate
enum class Prec { F64, F32, F32FB };

template <Prec P>
struct PrecTraits;
template <>
struct PrecTraits<Prec::F64> {
  using V = double;
};
template <>
struct PrecTraits<Prec::F32> {
  using V = float;
};
template <>
struct PrecTraits<Prec::F32FB> {
  using V = float;
};

// Node coordinate sources: [n][3] as given, or padded [n][4] (one aligned 32-byte
// record per node, so each random gather touches a single cache line).
struct NodesXYZ {
  const double* __restrict__ p;
  __device__ __forceinline__ void get(int32_t n, double (&x)[3]) const {
    const double* q = p + (int64_t)n * 3;
    x[0] = q[0];
    x[1] = q[1];
    x[2] = q[2];
  }
};
struct NodesPadded {
  const double4* __restrict__ p;
  __device__ __forceinline__ void get(int32_t n, double (&x)[3]) const {
    const double4 v = p[n];
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
  }
};

__global__ void k_pad_coords(const double* __restrict__ c, int64_t n, double4* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = make_double4(c[3 * i], c[3 * i + 1], c[3 * i + 2], 0.0);
}

// Coordinates of the element's nodes, gathered once into registers.
template <int NEN, typename NODES>
__device__ __forceinline__ void gather_nodes(const NODES& nodes, const int32_t (&E)[NEN], double (&Xn)[NEN][3]) {
#pragma unroll
  for (int a = 0; a < NEN; ++a) nodes.get(E[a], Xn[a]);
}

// Integrate one element from its gathered node coordinates Xn and coefficient c into k
// (value type V, c applied).  Adds flag bits to *f and counts a fallback in *fb.
template <int NEN, Prec P, Op OP = Op::Stiffness>
__device__ __forceinline__ void element_values_at(const double (&Xn)[NEN][3], double c, float tau,
                                                  typename PrecTraits<P>::V (&k)[ElemTraits<NEN>::T], uint32_t* f,
                                                  uint32_t* fb) {
  constexpr int T = ElemTraits<NEN>::T;
  using V = typename PrecTraits<P>::V;
  bool ok;
  if constexpr (P == Prec::F64) {
    double X[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) X[a][j] = a ? Xn[a][j] - Xn[0][j] : 0.0;
    ok = integrate<NEN, double, double, false, OP>(X, k, 0.0, nullptr);
  } else {
    float X[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) X[a][j] = a ? (float)(Xn[a][j] - Xn[0][j]) : 0.f;
    bool need_fb = false;
    ok = integrate<NEN, float, float, P == Prec::F32FB, OP>(X, k, tau, &need_fb);
    if constexpr (P == Prec::F32FB) {
      if (need_fb) {
        // Jacobian, determinant and adjugate in FP64 for this element
        double Xd[NEN][3];
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
          for (int j = 0; j < 3; ++j) Xd[a][j] = a ? Xn[a][j] - Xn[0][j] : 0.0;
        ok = integrate<NEN, double, float, false, OP>(Xd, k, 0.0, nullptr);
        *fb += 1;
      }
    }
  }
  bool finite = true;
#pragma unroll
  for (int p = 0; p < T; ++p) {
    k[p] = (V)(c * (double)k[p]);
    finite = finite && isfinite((double)k[p]);
  }
  if (!ok) *f |= KB_F_INVERTED;
  if (!finite) *f |= KB_F_NONFINITE;
}

// Gather and integrate element e.  E must be valid.  Each node's offset from node 0 is
// formed as soon as it arrives, so at most two nodes' FP64 coordinates are live.
template <int NEN, Prec P, typename NODES, Op OP = Op::Stiffness>
__device__ __forceinline__ void element_values(const NODES& nodes, const double* __restrict__ coef, int64_t e,
                                               const int32_t (&E)[NEN], float tau,
                                               typename PrecTraits<P>::V (&k)[ElemTraits<NEN>::T], uint32_t* f,
                                               uint32_t* fb) {
  constexpr int T = ElemTraits<NEN>::T;
  using V = typename PrecTraits<P>::V;
  double X0[3];
  nodes.get(E[0], X0);
  const double c = coef[e];
  bool ok;
  if constexpr (P == Prec::F64) {
    double X[NEN][3];
    X[0][0] = X[0][1] = X[0][2] = 0.0;
#pragma unroll
    for (int a = 1; a < NEN; ++a) {
      double xa[3];
      nodes.get(E[a], xa);
#pragma unroll
      for (int j = 0; j < 3; ++j) X[a][j] = xa[j] - X0[j];
    }
    ok = integrate<NEN, double, double, false, OP>(X, k, 0.0, nullptr);
  } else {
    float X[NEN][3];
    X[0][0] = X[0][1] = X[0][2] = 0.f;
#pragma unroll
    for (int a = 1; a < NEN; ++a) {
      double xa[3];
      nodes.get(E[a], xa);
#pragma unroll
      for (int j = 0; j < 3; ++j) X[a][j] = (float)(xa[j] - X0[j]);
    }
    bool need_fb = false;
    ok = integrate<NEN, float, float, P == Prec::F32FB, OP>(X, k, tau, &need_fb);
    if constexpr (P == Prec::F32FB) {
      if (need_fb) {
        // Jacobian, determinant and adjugate in FP64 for this element (nodes re-read)
        double Xd[NEN][3];
        Xd[0][0] = Xd[0][1] = Xd[0][2] = 0.0;
#pragma unroll
        for (int a = 1; a < NEN; ++a) {
          double xa[3];
          nodes.get(E[a], xa);
#pragma unroll
          for (int j = 0; j < 3; ++j) Xd[a][j] = xa[j] - X0[j];
        }
        ok = integrate<NEN, double, float, false, OP>(Xd, k, 0.0, nullptr);
        *fb += 1;
      }
    }
  }
  bool finite = true;
#pragma unroll
  for (int p = 0; p < T; ++p) {
    k[p] = (V)(c * (double)k[p]);
    finite = finite && isfinite((double)k[p]);
  }
  if (!ok) *f |= KB_F_INVERTED;
  if (!finite) *f |= KB_F_NONFINITE;
}

// A brick integrated by a lane pair (lanes 2i and 2i+1; h = lane & 1): lane h gathers
// nodes 4h .. 4h+3, the coordinates relative to node 0 are exchanged by shuffles, each
// lane integrates the four points of its half of the rule and the two halves of k are
// added.  Both lanes of a pair must be active together; both end with the same k and
// flags (the fallback is counted once, by h = 0).
template <Prec P>
__device__ __forceinline__ void element_values_pair(const NodesPadded& nodes, const double* __restrict__ coef,
                                                    int64_t e, const int32_t (&E)[8], float tau, int h,
                                                    typename PrecTraits<P>::V (&k)[36], uint32_t* f, uint32_t* fb) {
  using V = typename PrecTraits<P>::V;
  double xo[4][3];  // (a branch per half keeps every index into E a constant)
  if (h) {
#pragma unroll
    for (int a = 0; a < 4; ++a) nodes.get(E[4 + a], xo[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a) nodes.get(E[a], xo[a]);
  }
  double X0[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double other = __shfl_xor(xo[0][j], 1, 64);
    X0[j] = h ? other : xo[0][j];
  }
  double Xd[8][3];  // all eight nodes relative to node 0: own half and the partner's
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double mine = xo[a][j] - X0[j];
      const double other = __shfl_xor(mine, 1, 64);
      Xd[a][j] = h ? other : mine;
      Xd[4 + a][j] = h ? mine : other;
    }
  const double c = coef[e];
  bool ok;
  if constexpr (P == Prec::F64) {
    ok = hex_integrate_half<double, double, false>(Xd, k, 0.0, nullptr, h);
  } else {
    float X[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) X[a][j] = (float)Xd[a][j];
    bool need_fb = false;
    ok = hex_integrate_half<float, float, P == Prec::F32FB>(X, k, tau, &need_fb, h);
    if constexpr (P == Prec::F32FB) {
      need_fb = need_fb || (__shfl_xor((int)need_fb, 1, 64) != 0);
      if (need_fb) {  // the whole element, both halves, with FP64 geometry
        ok = hex_integrate_half<double, float, false>(Xd, k, 0.0, nullptr, h);
        if (h == 0) *fb += 1;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 36; ++p) k[p] += __shfl_xor(k[p], 1, 64);
  ok = ok && (__shfl_xor((int)ok, 1, 64) != 0);
  bool finite = true;
#pragma unroll
  for (int p = 0; p < 36; ++p) {
    k[p] = (V)(c * (double)k[p]);
    finite = finite && isfinite((double)k[p]);
  }
  if (!ok) *f |= KB_F_INVERTED;
  if (!finite) *f |= KB_F_NONFINITE;
}

template <int NEN, Prec P, Op OP = Op::Stiffness>
__global__ __launch_bounds__(256) void k_integrate_store(const int32_t* __restrict__ conn,
                                                         const double* __restrict__ coords,
                                                         const double* __restrict__ coef, int64_t n_elem,
                                                         int64_t n_node, float tau,
                                                         typename PrecTraits<P>::V* __restrict__ out,
                                                         uint32_t* __restrict__ status) {
  constexpr int T = ElemTraits<NEN>::T;
  using V = typename PrecTraits<P>::V;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  int32_t E[NEN];
  load_conn<NEN>(conn, e, E);
  uint32_t f = check_conn<NEN>(E, n_node);
  V k[T];
  uint32_t fb = 0;
  if (f) {
#pragma unroll
    for (int p = 0; p < T; ++p) k[p] = V(0);
  } else {
    element_values<NEN, P, NodesXYZ, OP>(NodesXYZ{coords}, coef, e, E, tau, k, &f, &fb);
  }
#pragma unroll
  for (int p = 0; p < T; ++p) out[e * T + p] = k[p];
  if (f) raise_flag(status, f);
  if (fb) atomicAdd(&status[1], fb);
}

// ------------------------------------------------------------------- row reduce
template <typename V>
struct Bits;
template <>
struct Bits<double> {
  using U = uint64_t;
  __device__ static U get(double v) { return (U)__double_as_longlong(v); }
};
template <>
struct Bits<float> {
  using U = uint32_t;
  __device__ static U get(float v) { return __float_as_uint(v); }
};

}  // namespace kb
