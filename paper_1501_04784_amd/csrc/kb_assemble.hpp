// kb_assemble.hpp -- atomic-free assembly of lower-triangular CSR K on gfx950.
//
// Every element contributes nen(nen+1)/2 lower pairs (Alg. 1 mapping): the node of
// rank r in its element (by global id) owns the r+1 pairs (itself, smaller ids) whose
// global row is that node.  Assembly (Eq. 6) sums the pairs with equal (row, col).
//
// Data movement: two partition passes, then a streaming reduction in LDS.
//   hist     per tile of elements: pairs per row bucket (row >> s1), tile-major.
//   offsets  transpose + exclusive scan + transpose back: each tile's write offset in
//            each bucket; bucket boundaries.
//   pass 1   per tile (one element per lane): integrate the element (or read given
//            values; coordinates come from a padded 32-byte-per-node copy made by
//            k_pad_coords), stage its pairs in LDS grouped by bucket, write each bucket's run
//            at the tile's offset as (row, col, value) arrays.  Also the largest value
//            exponent, which fixes the exact-sum scale below.
//   pass 2   per fixed-size segment of a bucket: histogram of sub-buckets
//            (row >> s2); per bucket, a prefix over its segments for each sub-bucket;
//            then LDS-staged scatter into contiguous sub-bucket ranges; pairs are
//            repacked as (row_local << colbits | col, value).
//   pass 3   per sub-bucket: stream its pairs into an LDS hash table keyed by the
//            packed (row, col); each value is added as a 128-bit fixed-point integer
//            (scale 2^F from the largest exponent), so every sum is exact and its
//            result does not depend on the order of the additions: the output is
//            bitwise deterministic although the partition passes order pairs through
//            LDS atomics.  Entries are then ordered by (row, col) and converted once
//            (correct rounding of the exact sum to FP64, then to the value type).
//   final    scan of per-sub-bucket unique counts; row_ptr and the compacted col/vals.
// A sub-bucket whose distinct entries overflow the table takes a slow single-lane path
// in global memory (heap sort, then the same exact sums).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kb_element.hpp"
#include "kb_kernels.hpp"
#include "kbuild.h"

namespace kb {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;  // packed keys never use bit 31

// ----------------------------------------------------------------- block helpers
// exclusive scan of one uint32 per thread across the block; *total = block sum.
// smem must hold (blockDim/64 + 1) words.  Contains barriers: call from all threads.
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t* smem, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) smem[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < nw; ++w) {
      uint32_t t = smem[w];
      smem[w] = s;
      s += t;
    }
    smem[nw] = s;
  }
  __syncthreads();
  const uint32_t r = x - v + smem[wave];
  *total = smem[nw];
  __syncthreads();
  return r;
}

// in-place exclusive scan of a[0..n) in LDS (n arbitrary); returns the total.
template <typename T>
__device__ __forceinline__ uint32_t block_scan_array(T* a, int n, uint32_t* smem) {
  const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int lo = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i)
    if (lo + i < n) s += (uint32_t)a[lo + i];
  uint32_t total;
  uint32_t off = block_scan_u32(s, smem, &total);
  for (int i = 0; i < per; ++i)
    if (lo + i < n) {
      const uint32_t v = (uint32_t)a[lo + i];
      a[lo + i] = (T)off;
      off += v;
    }
  __syncthreads();
  return total;
}

// ------------------------------------------------------- exact fixed-point sums
// A finite double v is m * 2^(E-1075) (m < 2^53).  With the scale F = 1117 - Emax,
// where Emax is the largest biased exponent of all values, q = v * 2^F is below 2^95
// in magnitude, so up to 2^31 of them sum exactly in a 128-bit two's complement
// integer.  Bits below 2^-F are dropped (truncation toward zero, independent of
// order).  Non-finite values contribute 0 (they are flagged elsewhere).
__device__ __forceinline__ int biased_exponent(double v) {
  return (int)((__double_as_longlong(v) >> 52) & 0x7FF);
}

__device__ __forceinline__ void to_fixed(double v, int F, uint64_t& lo, uint64_t& hi) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  int E = (int)((b >> 52) & 0x7FF);
  uint64_t m = b & ((1ull << 52) - 1);
  lo = 0;
  hi = 0;
  if (E == 0x7FF) return;
  if (E == 0)
    E = 1;  // subnormal
  else
    m |= 1ull << 52;
  if (m == 0) return;
  const int sh = E - 1075 + F;
  if (sh >= 64) {
    hi = m << (sh - 64);
  } else if (sh > 0) {
    lo = m << sh;
    hi = m >> (64 - sh);
  } else if (sh == 0) {
    lo = m;
  } else if (sh > -64) {
    lo = m >> (-sh);
  }
  if (b >> 63) {  // negate (two's complement)
    lo = ~lo + 1;
    hi = ~hi + (lo == 0 ? 1ull : 0ull);
  }
}

// q (two's complement 128-bit, |q| < 2^95) as c0 + c1 * 2^48 with c0 in [0, 2^48)
// and c1 signed: sums of up to 2^16 such terms fit in one unsigned / signed 64-bit
// word each, so they can be accumulated without carries (and in any order).
__device__ __forceinline__ void split48(uint64_t lo, uint64_t hi, uint64_t& c0, int64_t& c1) {
  c0 = lo & ((1ull << 48) - 1);
  c1 = (int64_t)((lo >> 48) | (hi << 16));
}

// split48 chunks of trunc(v * 2^F) for a double or float value (non-finite: zero),
// formed in FP64 arithmetic, where every step is exact: v 2^F only moves the exponent
// (|q| < 2^95; a result below 2^-1022 truncates to 0 either way), trunc and floor give
// integers, and c1 = floor(q / 2^48), c0 = q - c1 2^48 in [0, 2^48) are multiples of
// q's last bit below 2^53 of it.  Each integer then becomes a 64-bit word by an exact
// FP64 addition: c0 + 2^52 and c1 + 1.5 2^52 (|c1| < 2^47) lie in [2^52, 2^53), where
// the spacing is 1, so their bit patterns are those of the constants plus the integer
// (two's complement for a negative c1), and the constants' low 32 bits are zero: one
// 32-bit subtraction from the high word leaves the integer.  The same integers as
// split48 of to_fixed's q, without forming the 128-bit integer and without branches.
__device__ __forceinline__ void to_chunks(double v, int F, uint64_t& c0, int64_t& c1) {
  const double d = isfinite(v) ? v : 0.0;
  const double q = trunc(ldexp(d, F));
  const double h = floor(ldexp(q, -48));
  const double l = fma(h, -0x1p48, q);  // [0, 2^48)
  const uint64_t bl = (uint64_t)__double_as_longlong(l + 0x1p52);
  const uint64_t bh = (uint64_t)__double_as_longlong(h + 0x1.8p52);
  c0 = bl - 0x4330000000000000ull;
  c1 = (int64_t)(bh - 0x4338000000000000ull);
}
__device__ __forceinline__ void to_chunks(float v, int F, uint64_t& c0, int64_t& c1) {
  to_chunks((double)v, F, c0, c1);  // a float is exactly a double
}

// chunk sums back to the exact 128-bit value
__device__ __forceinline__ void join48(uint64_t s0, int64_t s1, uint64_t& lo, uint64_t& hi) {
  const uint64_t a_lo = (uint64_t)s1 << 48;
  const uint64_t a_hi = (uint64_t)(s1 >> 16);  // arithmetic shift keeps the sign
  lo = s0 + a_lo;
  hi = a_hi + (lo < s0 ? 1ull : 0ull);
}

// exact 128-bit value -> V (double or float), rounded once to nearest; then scaled by
// 2^-F (exact unless the result is subnormal).  The 64 leading bits carry a sticky bit
// for the rest, so the one rounding of the 64-bit integer to V is that of the whole.
template <typename V>
__device__ __forceinline__ V from_fixed_as(uint64_t lo, uint64_t hi, int F) {
  const bool neg = (int64_t)hi < 0;
  if (neg) {
    lo = ~lo + 1;
    hi = ~hi + (lo == 0 ? 1ull : 0ull);
  }
  uint64_t top = lo;
  int sh = 0;
  if (hi != 0) {
    const int lz = __clzll((long long)hi);
    top = lz ? ((hi << lz) | (lo >> (64 - lz))) : hi;
    const uint64_t rest = lz ? (lo << lz) : lo;
    top |= rest ? 1ull : 0ull;  // sticky bit: 64 > 53 + 2 bits, so the rounding stays correct
    sh = 64 - lz;
  }
  V d;
  if constexpr (sizeof(V) == 8)
    d = ldexp(ldexp((double)top, sh), -F);
  else
    d = ldexpf(ldexpf((float)top, sh), -F);
  return neg ? -d : d;
}
__device__ __forceinline__ double from_fixed(uint64_t lo, uint64_t hi, int F) {
  return from_fixed_as<double>(lo, hi, F);
}

// What V's rounding h of an exact value left out, rounded to V: h + residual holds the
// value to about twice V's precision.  h * 2^F is an integer (the value rounded), so its
// fixed-point form is exact and the difference is exact before its one rounding.
template <typename V>
__device__ __forceinline__ V fixed_residual(uint64_t lo, uint64_t hi, int F, V h) {
  uint64_t a, b;
  to_fixed((double)h, F, a, b);
  const uint64_t dl = lo - a;
  const uint64_t dh = hi - b - (lo < a ? 1ull : 0ull);
  return from_fixed_as<V>(dl, dh, F);
}

// ---------------------------------------------------------------------- histogram
// Per tile of `te` elements: pairs per bucket (row >> s1), written tile-major
// hist[t * nb + b].  Flags index errors; invalid elements contribute nothing.
// Reserve the pairs of local rows OFF .. OFF+N-1 of an element in their buckets' LDS
// counters: each run of consecutive rows in one bucket takes one atomic for its total
// (under a natural numbering an element's neighbouring nodes mostly share a bucket, and
// per-row increments from neighbouring lanes would serialise on one address); a row
// after the first of its run starts where its predecessor's pairs end.  q: first place
// of each row's r+1 pairs within the bucket's part of the tile.
template <int N, int OFF, int NE>
__device__ __forceinline__ void reserve_rows(uint32_t* cnt, const int32_t (&E)[NE], const int (&r)[NE], int s1,
                                             uint32_t (&q)[N]) {
  uint32_t tot[N];  // pairs from row a to the end of its run
  tot[N - 1] = (uint32_t)(r[OFF + N - 1] + 1);
#pragma unroll
  for (int a = N - 2; a >= 0; --a)
    tot[a] = (uint32_t)(r[OFF + a] + 1) + ((E[OFF + a] >> s1) == (E[OFF + a + 1] >> s1) ? tot[a + 1] : 0u);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    if (a > 0 && (E[OFF + a] >> s1) == (E[OFF + a - 1] >> s1))
      q[a] = q[a - 1] + (uint32_t)(r[OFF + a - 1] + 1);
    else
      q[a] = atomicAdd(&cnt[E[OFF + a] >> s1], tot[a]);
  }
}

template <int NEN>
__global__ __launch_bounds__(256) void k_hist_buckets(const int32_t* __restrict__ conn, int64_t n_elem, int64_t n_node,
                                                      int te, int s1, int nb, uint32_t* __restrict__ hist,
                                                      uint32_t* __restrict__ status) {
  extern __shared__ uint32_t s_h[];  // [nb]
  const int64_t t = blockIdx.x;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s_h[b] = 0;
  __syncthreads();
  const int64_t e0 = t * te, e1 = (e0 + te < n_elem) ? e0 + te : n_elem;
  uint32_t flags = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    int32_t E[NEN];
    load_conn<NEN>(conn, e, E);
    const uint32_t f = check_conn<NEN>(E, n_node);
    if (f) {
      flags |= f;
      continue;
    }
    int r[NEN];
    node_ranks<NEN>(E, r);
    uint32_t q[NEN];
    reserve_rows<NEN, 0>(s_h, E, r, s1, q);
  }
  if (flags) raise_flag(status, flags);
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[t * nb + b] = s_h[b];
}

// Tile offsets from the tile-major histogram hist[t][b] (tiles x buckets) without
// transposing it: column sums over chunks of kColChunk tiles, a scan of those per bucket,
// then each chunk's columns walked again, counts turned into offsets in place:
// hist[t][b] = bstart[b] + (pairs of bucket b in tiles before t).
constexpr int kColChunk = 64;

// grid (chunks, ceil(nb / 256)): csum[c][b] = sum of hist[t][b] over the tiles of chunk c
__global__ __launch_bounds__(256) void k_col_chunks(const uint32_t* __restrict__ hist, int64_t ntiles, int nb,
                                                    uint32_t* __restrict__ csum) {
  const int64_t c = blockIdx.x;
  const int b = blockIdx.y * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t t0 = c * kColChunk, t1 = t0 + kColChunk < ntiles ? t0 + kColChunk : ntiles;
  uint32_t sum = 0;
#pragma unroll 8
  for (int64_t t = t0; t < t1; ++t) sum += hist[t * nb + b];
  csum[c * nb + b] = sum;
}

// one workgroup per bucket b: exclusive scan of csum[.][b] over the chunks, in place; the
// bucket's total to tot[b]
__global__ __launch_bounds__(256) void k_col_scan(uint32_t* __restrict__ csum, int64_t nchunk, int nb,
                                                  uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_scan[8];
  const int b = blockIdx.x;
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < nchunk; c0 += blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    const uint32_t v = c < nchunk ? csum[c * nb + b] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_u32(v, s_scan, &total);
    if (c < nchunk) csum[c * nb + b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tot[b] = carry;
}

// grid (chunks, ceil(nb / 256)): counts of chunk c turned into offsets in place
__global__ __launch_bounds__(256) void k_col_offsets(uint32_t* __restrict__ hist, const uint32_t* __restrict__ csum,
                                                     const uint32_t* __restrict__ bstart, int64_t ntiles, int nb) {
  const int64_t c = blockIdx.x;
  const int b = blockIdx.y * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  uint32_t run = bstart[b] + csum[c * nb + b];
  const int64_t t0 = c * kColChunk, t1 = t0 + kColChunk < ntiles ? t0 + kColChunk : ntiles;
#pragma unroll 8
  for (int64_t t = t0; t < t1; ++t) {
    const uint32_t v = hist[t * nb + b];
    hist[t * nb + b] = run;
    run += v;
  }
}

// single block: segbase[b] = number of pass-2 segments in buckets before b
// (segbase[nb] = total), a bucket of n pairs having ceil(n / seg) segments
__global__ __launch_bounds__(256) void k_segments(const uint32_t* __restrict__ bstart, int nb, int seg,
                                                  uint32_t* __restrict__ segbase) {
  __shared__ uint32_t s_scan[8];
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int b = b0 + threadIdx.x;
    const uint32_t n = (b < nb) ? (bstart[b + 1] - bstart[b] + seg - 1) / seg : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_u32(n, s_scan, &total);
    if (b < nb) segbase[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) segbase[nb] = carry;
}

// ------------------------------------------------------------------------ pass 1
// A tile is BLOCK elements, one per lane.  Its pairs are grouped by bucket (row >> s1)
// in LDS and each bucket's run is written at the tile's offset in that bucket.
template <typename V, int BLOCK>
struct Pass1Smem {
  uint64_t* key;  // [cap] staged (row << 32 | col)
  V* val;         // [cap] staged values
  uint32_t* cnt;  // [nb] pairs per bucket, then local run starts
  uint32_t* base; // [nb] global offset of this tile in bucket b
  uint32_t* scan; // [BLOCK/64 + 1]
  uint32_t* emax; // [1]
  __device__ Pass1Smem(unsigned char* smem, int cap, int nb) {
    key = (uint64_t*)smem;
    val = (V*)(key + cap);
    cnt = (uint32_t*)(val + cap);
    base = cnt + nb;
    scan = base + nb;
    emax = scan + (BLOCK / 64 + 1);
  }
};

// count the tile's pairs per bucket, keeping each (element, row) group's offset
// within its bucket in q; then scan: sm.cnt = local run starts.  Returns the tile's
// pair count.  Block-wide (barriers).
template <int NEN, typename SM>
__device__ __forceinline__ uint32_t pass1_count(const SM& sm, const int32_t (&E)[NEN], const int (&r)[NEN], bool valid,
                                                int s1, int nb, uint32_t (&q)[NEN]) {
  if (valid) reserve_rows<NEN, 0>(sm.cnt, E, r, s1, q);
  __syncthreads();
  return block_scan_array(sm.cnt, nb, sm.scan);
}

// stage one element's pairs: the r+1 pairs of row E[a] go contiguously into its bucket
template <int NEN, typename V, typename SM>
__device__ __forceinline__ void pass1_stage(const SM& sm, const int32_t (&E)[NEN], const uint32_t (&q)[NEN],
                                            const V (&k)[ElemTraits<NEN>::T], int s1) {
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    uint32_t pos = sm.cnt[E[a] >> s1] + q[a];
    const uint64_t rk = (uint64_t)(uint32_t)E[a] << 32;
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
      if (E[b] <= E[a]) {
        sm.key[pos] = rk | (uint32_t)E[b];
        sm.val[pos] = (a >= b) ? k[lidx(a, b)] : k[lidx(b, a)];
        ++pos;
      }
    }
  }
}

// write the staged pairs: index i lies in bucket b = row >> s1, local start sm.cnt[b]
template <typename V, typename SM>
__device__ __forceinline__ void pass1_write(const SM& sm, uint32_t n_items, int s1, int nthreads,
                                            uint16_t* __restrict__ orow, uint32_t* __restrict__ ocol,
                                            V* __restrict__ oval) {
  for (uint32_t i = threadIdx.x; i < n_items; i += nthreads) {
    const uint64_t key = sm.key[i];
    const uint32_t row = (uint32_t)(key >> 32);
    const int b = (int)(row >> s1);
    const uint32_t g = sm.base[b] + (i - sm.cnt[b]);
    orow[g] = (uint16_t)(row & ((1u << s1) - 1));  // row within its bucket
    ocol[g] = (uint32_t)key;
    oval[g] = sm.val[i];
  }
}

// largest finite biased exponent of an element's values
template <int T, typename V>
__device__ __forceinline__ uint32_t values_emax(const V (&k)[T]) {
  uint32_t m = 0;
#pragma unroll
  for (int p = 0; p < T; ++p) {
    const uint32_t ep = (uint32_t)biased_exponent((double)k[p]);
    m = (ep > m && ep < 0x7FF) ? ep : m;
  }
  return m;
}

// element values from given per-element lower triangles (assembly-only path)
template <int T, typename V>
__device__ __forceinline__ void read_values(const V* __restrict__ klow, int64_t e, V (&k)[T], uint32_t* flags) {
  bool finite = true;
#pragma unroll
  for (int p = 0; p < T; ++p) {
    k[p] = klow[e * T + p];
    finite = finite && isfinite((double)k[p]);
  }
  if (!finite) *flags |= KB_F_NONFINITE;
}

// Bricks: one tile per workgroup; tiles are assigned XCD-contiguously, so the runs that
// neighbouring tiles write side by side meet in one L2.  OP: the integrand (unless the
// values are given).
template <int NEN, Prec P, bool FROM_VALUES, int BLOCK, Op OP = Op::Stiffness>
__global__ __launch_bounds__(BLOCK) void k_pass1(const int32_t* __restrict__ conn, const double4* __restrict__ coords4,
                                               const double* __restrict__ coef,
                                               const typename PrecTraits<P>::V* __restrict__ klow, int64_t n_elem,
                                               int64_t n_node, float tau, int s1, int nb, int64_t ntiles,
                                               const uint32_t* __restrict__ off1, uint16_t* __restrict__ orow,
                                               uint32_t* __restrict__ ocol, typename PrecTraits<P>::V* __restrict__ oval,
                                               uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  using V = typename PrecTraits<P>::V;
  constexpr int T = ElemTraits<NEN>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, BLOCK> sm(smem, BLOCK * T, nb);
  const int64_t t = xcd_item(blockIdx.x, gridDim.x);
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    sm.cnt[b] = 0;
    sm.base[b] = off1[t * nb + b];
  }
  if (threadIdx.x == 0) *sm.emax = 0;
  __syncthreads();
  const int64_t e = t * BLOCK + threadIdx.x;
  int32_t E[NEN];
  bool valid = false;
  if (e < n_elem) {
    load_conn<NEN>(conn, e, E);
    valid = check_conn<NEN>(E, n_node) == 0;
  }
  int r[NEN];
  uint32_t q[NEN];
  if (valid) node_ranks<NEN>(E, r);
  const uint32_t n_items = pass1_count<NEN>(sm, E, r, valid, s1, nb, q);
  uint32_t flags = 0, fb = 0;
  if (valid) {
    V k[T];
    if constexpr (FROM_VALUES)
      read_values<T>(klow, e, k, &flags);
    else
      element_values<NEN, P, NodesPadded, OP>(NodesPadded{coords4}, coef, e, E, tau, k, &flags, &fb);
    atomicMax(sm.emax, values_emax<T>(k));
    pass1_stage<NEN>(sm, E, q, k, s1);
  }
  if (flags) raise_flag(status, flags);
  if (fb) atomicAdd(&status[1], fb);
  __syncthreads();
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
  pass1_write(sm, n_items, s1, BLOCK, orow, ocol, oval);
}

// Bricks in FP64 from coordinates (one element per lane at the register limit): two
// tiles per workgroup of 2 BLOCK lanes, so that each SIMD holds two waves while the
// elements are gathered and integrated.  The two tiles are then counted, staged and
// written one after the other through the one staging area (BLOCK elements' pairs).
// Workgroup w takes tiles 2w and 2w + 1, XCD-contiguously as k_pass1.
template <int NEN, Prec P, int BLOCK, Op OP = Op::Stiffness>
__global__ __launch_bounds__(2 * BLOCK) void k_pass1_two(const int32_t* __restrict__ conn,
                                                       const double4* __restrict__ coords4,
                                                       const double* __restrict__ coef, int64_t n_elem, int64_t n_node,
                                                       float tau, int s1, int nb, int64_t ntiles,
                                                       const uint32_t* __restrict__ off1, uint16_t* __restrict__ orow,
                                                       uint32_t* __restrict__ ocol,
                                                       typename PrecTraits<P>::V* __restrict__ oval,
                                                       uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  using V = typename PrecTraits<P>::V;
  constexpr int T = ElemTraits<NEN>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, 2 * BLOCK> sm(smem, BLOCK * T, nb);
  const int64_t w = xcd_item(blockIdx.x, gridDim.x);
  const int half = threadIdx.x >= BLOCK ? 1 : 0;
  const int64_t e = (2 * w + half) * BLOCK + (threadIdx.x - half * BLOCK);
  if (threadIdx.x == 0) *sm.emax = 0;
  int32_t E[NEN];
  bool valid = false;
  if (e < n_elem) {
    load_conn<NEN>(conn, e, E);
    valid = check_conn<NEN>(E, n_node) == 0;
  }
  int r[NEN];
  if (valid) node_ranks<NEN>(E, r);
  uint32_t flags = 0, fb = 0;
  V k[T];
  if (valid) element_values<NEN, P, NodesPadded, OP>(NodesPadded{coords4}, coef, e, E, tau, k, &flags, &fb);
  if (flags) raise_flag(status, flags);
  if (fb) atomicAdd(&status[1], fb);
  __syncthreads();
  if (valid) atomicMax(sm.emax, values_emax<T>(k));
  for (int h = 0; h < 2; ++h) {
    const int64_t t = 2 * w + h;
    if (t >= ntiles) break;
    for (int b = threadIdx.x; b < nb; b += 2 * BLOCK) {
      sm.cnt[b] = 0;
      sm.base[b] = off1[t * nb + b];
    }
    __syncthreads();
    uint32_t q[NEN];
    const bool mine = valid && half == h;
    if (mine) reserve_rows<NEN, 0>(sm.cnt, E, r, s1, q);
    __syncthreads();
    const uint32_t n_items = block_scan_array(sm.cnt, nb, sm.scan);
    if (mine) pass1_stage<NEN>(sm, E, q, k, s1);
    __syncthreads();
    pass1_write(sm, n_items, s1, 2 * BLOCK, orow, ocol, oval);
    __syncthreads();  // the staging area is reused by the next tile
  }
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
}

// stage the pairs of rows R0 .. R0+3 of a brick (the lane's half of a lane pair)
template <int R0, typename V, typename SM>
__device__ __forceinline__ void pair_stage_half(const SM& sm, const int32_t (&E)[8], const uint32_t (&q)[4],
                                                const V (&k)[36], int s1) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = R0 + a;
    uint32_t pos = sm.cnt[E[row] >> s1] + q[a];
    const uint64_t rk = (uint64_t)(uint32_t)E[row] << 32;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (E[b] <= E[row]) {
        sm.key[pos] = rk | (uint32_t)E[b];
        sm.val[pos] = row >= b ? k[lidx(row, b)] : k[lidx(b, row)];
        ++pos;
      }
    }
  }
}

// Bricks, stiffness matrix: a lane pair per element (element_values_pair), BLOCK lanes
// and BLOCK / 2 elements per tile.  Twice the waves of one lane per element for the same
// staging LDS, and half the quadrature per lane; lane h counts and stages the pairs of
// rows 4h .. 4h+3.
template <Prec P, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pass1_pair(const int32_t* __restrict__ conn,
                                                    const double4* __restrict__ coords4,
                                                    const double* __restrict__ coef, int64_t n_elem, int64_t n_node,
                                                    float tau, int s1, int nb, const uint32_t* __restrict__ off1,
                                                    uint16_t* __restrict__ orow, uint32_t* __restrict__ ocol,
                                                    typename PrecTraits<P>::V* __restrict__ oval,
                                                    uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  using V = typename PrecTraits<P>::V;
  constexpr int NEN = 8, T = ElemTraits<NEN>::T, TE = BLOCK / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, BLOCK> sm(smem, TE * T, nb);
  const int64_t t = xcd_item(blockIdx.x, gridDim.x);
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    sm.cnt[b] = 0;
    sm.base[b] = off1[t * nb + b];
  }
  if (threadIdx.x == 0) *sm.emax = 0;
  __syncthreads();
  const int h = (int)(threadIdx.x & 1);
  const int64_t e = t * TE + (threadIdx.x >> 1);
  int32_t E[NEN];
  bool valid = false;
  if (e < n_elem) {
    load_conn<NEN>(conn, e, E);
    valid = check_conn<NEN>(E, n_node) == 0;
  }
  // offsets of the lane's four rows in their buckets (a branch per half keeps every
  // index into E and r a constant)
  uint32_t q[4];
  if (valid) {
    int r[NEN];
    node_ranks<NEN>(E, r);
    if (h) {
#pragma unroll
      for (int a = 0; a < 4; ++a) q[a] = atomicAdd(&sm.cnt[E[4 + a] >> s1], (uint32_t)(r[4 + a] + 1));
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) q[a] = atomicAdd(&sm.cnt[E[a] >> s1], (uint32_t)(r[a] + 1));
    }
  }
  __syncthreads();
  const uint32_t n_items = block_scan_array(sm.cnt, nb, sm.scan);
  uint32_t flags = 0, fb = 0;
  if (valid) {
    V k[T];
    element_values_pair<P>(NodesPadded{coords4}, coef, e, E, tau, h, k, &flags, &fb);
    atomicMax(sm.emax, values_emax<T>(k));
    if (h)
      pair_stage_half<4>(sm, E, q, k, s1);
    else
      pair_stage_half<0>(sm, E, q, k, s1);
  }
  if (flags) raise_flag(status, flags);
  if (fb) atomicAdd(&status[1], fb);
  __syncthreads();
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
  pass1_write(sm, n_items, s1, BLOCK, orow, ocol, oval);
}

// Tetrahedra: persistent workgroups.  XCD x owns one contiguous range of tiles and its
// workgroups walk it interleaved (neighbouring runs again meet in one L2).  The next
// tile's connectivity is loaded while the current tile is integrated, and its node
// coordinates while the current tile is written.
template <Prec P, bool FROM_VALUES, int BLOCK, Op OP = Op::Stiffness>
__global__ __launch_bounds__(BLOCK) void k_pass1_tet(const int32_t* __restrict__ conn,
                                                   const double4* __restrict__ coords4,
                                                   const double* __restrict__ coef,
                                                   const typename PrecTraits<P>::V* __restrict__ klow, int64_t n_elem,
                                                   int64_t n_node, float tau, int s1, int nb, int64_t ntiles,
                                                   const uint32_t* __restrict__ off1, uint16_t* __restrict__ orow,
                                                   uint32_t* __restrict__ ocol,
                                                   typename PrecTraits<P>::V* __restrict__ oval,
                                                   uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  using V = typename PrecTraits<P>::V;
  constexpr int NEN = 4, T = ElemTraits<NEN>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, BLOCK> sm(smem, BLOCK * T, nb);
  const int64_t G = gridDim.x, x = blockIdx.x % kXcds, w = blockIdx.x / kXcds;
  const int64_t nw = G / kXcds + (x < G % kXcds ? 1 : 0);
  const int64_t lo = x * (ntiles / kXcds) + min(x, ntiles % kXcds);
  const int64_t hi = lo + ntiles / kXcds + (x < ntiles % kXcds ? 1 : 0);
  int64_t t = lo + w;
  if (t >= hi) return;
  if (threadIdx.x == 0) *sm.emax = 0;

  auto fetch = [&](int64_t tt, int32_t (&Ef)[NEN]) {
    const int64_t e = tt * BLOCK + threadIdx.x;
    if (tt < hi && e < n_elem) {
      load_conn<NEN>(conn, e, Ef);
      return check_conn<NEN>(Ef, n_node) == 0;
    }
    return false;
  };
  int32_t E[NEN];
  bool valid = fetch(t, E);
  double Xn[NEN][3];
  double c_e = 0.0;
  if constexpr (!FROM_VALUES) {
    if (valid) {
      gather_nodes<NEN>(NodesPadded{coords4}, E, Xn);
      c_e = coef[t * BLOCK + threadIdx.x];
    }
  }
  uint32_t em = 0;  // largest value exponent seen by this lane
  while (true) {
    const int64_t e = t * BLOCK + threadIdx.x;
    for (int b = threadIdx.x; b < nb; b += BLOCK) {
      sm.cnt[b] = 0;
      sm.base[b] = off1[t * nb + b];
    }
    __syncthreads();
    int r[NEN];
    uint32_t q[NEN];
    if (valid) node_ranks<NEN>(E, r);
    const uint32_t n_items = pass1_count<NEN>(sm, E, r, valid, s1, nb, q);
    const int64_t tn = t + nw;
    int32_t En[NEN];
    const bool vn = fetch(tn, En);
    uint32_t flags = 0, fb = 0;
    if (valid) {
      V k[T];
      if constexpr (FROM_VALUES)
        read_values<T>(klow, e, k, &flags);
      else
        element_values_at<NEN, P, OP>(Xn, c_e, tau, k, &flags, &fb);
      const uint32_t me = values_emax<T>(k);
      em = me > em ? me : em;
      pass1_stage<NEN>(sm, E, q, k, s1);
    }
    if (flags) raise_flag(status, flags);
    if (fb) atomicAdd(&status[1], fb);
#pragma unroll
    for (int a = 0; a < NEN; ++a) E[a] = En[a];
    valid = vn;
    if constexpr (!FROM_VALUES) {
      if (valid) {
        gather_nodes<NEN>(NodesPadded{coords4}, E, Xn);
        c_e = coef[tn * BLOCK + threadIdx.x];
      }
    }
    __syncthreads();
    pass1_write(sm, n_items, s1, BLOCK, orow, ocol, oval);
    t = tn;
    if (t >= hi) break;
    __syncthreads();
  }
  if (em) atomicMax(sm.emax, em);
  __syncthreads();
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
}

// Elements of more than eight rows (nodes with several degrees of freedom), values
// given (assembly only).  A tile is `te` elements, few enough that their pairs fit in
// LDS; kWideThreads threads work on it:
//   - per (element, row a): the row's rank r_a among the element's ids, and its run of
//     r_a + 1 places in the tile's part of bucket E_a >> s1 (LDS counters);
//   - per pair, one thread each, values read in storage order (coalesced): pair (p, q)
//     belongs to the row of the larger id (a) and takes place rank(b) of that row's
//     run, b being the other corner (the diagonal takes the last place, r_a);
//   - the staged pairs, grouped by bucket, are written as runs (as for 4 and 8 rows).
constexpr int kWideThreads = 1024;  // threads per wide pass-1 workgroup (one per CU: LDS)

template <int NEN, typename V>
__global__ __launch_bounds__(kWideThreads) void k_pass1_wide(const int32_t* __restrict__ conn, const V* __restrict__ klow,
                                                  int64_t n_elem, int64_t n_node, int te, int s1, int nb,
                                                  const uint32_t* __restrict__ off1, uint16_t* __restrict__ orow,
                                                  uint32_t* __restrict__ ocol, V* __restrict__ oval,
                                                  uint32_t* __restrict__ emax, uint32_t* __restrict__ status) {
  constexpr int T = ElemTraits<NEN>::T, NT = kWideThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, NT> sm(smem, te * T, nb);
  int32_t* s_E = (int32_t*)(sm.emax + 1);    // [te * NEN] the tile's connectivity
  uint32_t* s_q = (uint32_t*)(s_E + te * NEN);  // [te * NEN] run offset of each row in its bucket
  uint32_t* s_rank = s_q + te * NEN;            // [te * NEN] rank of each corner's id
  uint32_t* s_ok = s_rank + te * NEN;           // [te] element valid
  uint16_t* s_pq = (uint16_t*)(s_ok + te);      // [T] packed index -> (p << 8 | q)
  const int64_t t = xcd_item(blockIdx.x, gridDim.x);
  const int64_t e0 = t * te;
  const int ne = (int)(n_elem - e0 < te ? n_elem - e0 : te);
  for (int b = threadIdx.x; b < nb; b += NT) {
    sm.cnt[b] = 0;
    sm.base[b] = off1[t * nb + b];
  }
  if (threadIdx.x == 0) *sm.emax = 0;
  for (int i = threadIdx.x; i < T; i += NT) {
    int p = 0;
    while ((p + 1) * (p + 2) / 2 <= i) ++p;
    s_pq[i] = (uint16_t)(p << 8 | (i - p * (p + 1) / 2));
  }
  for (int i = threadIdx.x; i < ne * NEN; i += NT) s_E[i] = conn[e0 * NEN + i];
  __syncthreads();
  uint32_t flags = 0;
  for (int el = threadIdx.x; el < ne; el += NT) {
    int32_t E[NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) E[a] = s_E[el * NEN + a];
    const uint32_t f = check_conn<NEN>(E, n_node);
    flags |= f;
    s_ok[el] = f == 0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ne * NEN; j += NT) {
    const int el = j / NEN;
    if (!s_ok[el]) continue;
    const int32_t Ea = s_E[j];
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < NEN; ++b) r += (s_E[el * NEN + b] < Ea) ? 1u : 0u;
    s_rank[j] = r;
    s_q[j] = atomicAdd(&sm.cnt[Ea >> s1], r + 1);
  }
  __syncthreads();
  const uint32_t n_items = block_scan_array(sm.cnt, nb, sm.scan);  // cnt: local run starts
  uint32_t em = 0;
  bool finite = true;
  const V* __restrict__ k = klow + e0 * T;
  for (int i = threadIdx.x; i < ne * T; i += NT) {
    const int el = i / T, kk = i - el * T;
    if (!s_ok[el]) continue;
    const uint32_t pq = s_pq[kk];
    const int p = (int)(pq >> 8), q = (int)(pq & 255u);
    const int32_t Ep = s_E[el * NEN + p], Eq = s_E[el * NEN + q];
    const bool up = Ep >= Eq;
    const int a = up ? p : q, b = up ? q : p;
    const int32_t Ea = up ? Ep : Eq, Eb = up ? Eq : Ep;
    const uint32_t pos = sm.cnt[Ea >> s1] + s_q[el * NEN + a] + s_rank[el * NEN + b];
    const V v = k[i];
    finite = finite && isfinite((double)v);
    const uint32_t ep = (uint32_t)biased_exponent((double)v);
    em = (ep > em && ep < 0x7FF) ? ep : em;
    sm.key[pos] = (uint64_t)(uint32_t)Ea << 32 | (uint32_t)Eb;
    sm.val[pos] = v;
  }
  if (!finite) flags |= KB_F_NONFINITE;
  if (flags) raise_flag(status, flags);
  if (em) atomicMax(sm.emax, em);
  __syncthreads();
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
  pass1_write(sm, n_items, s1, NT, orow, ocol, oval);
}

// ----------------------------------------------------- running sums as a source
// A grouped build carries the sums of the groups done so far as a lower CSR (entries in
// row order, with rows[], residuals res[] and nnz in device memory).  The next group's
// pass reads them back as pairs (row, col, value) and (row, col, residual) next to its
// elements' pairs.  Tiles of kCsrTile entries follow the element tiles.  The entries
// are read only if they were written (nnz <= cap); rows outside [0, n_node) are skipped
// (both kernels apply the same test, so counts and writes agree).
constexpr int kCsrTile = 2048;

__device__ __forceinline__ int64_t csr_entries(const int64_t* nnz_dev, int64_t cap) {
  const int64_t n = *nnz_dev;
  return (n >= 0 && n <= cap) ? n : 0;
}

__global__ __launch_bounds__(256) void k_hist_csr(const int32_t* __restrict__ rows, const int64_t* __restrict__ nnz_dev,
                                                  int64_t cap, int64_t n_node, int s1, int nb,
                                                  uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t s_h[];  // [nb]
  const int64_t t = blockIdx.x;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s_h[b] = 0;
  __syncthreads();
  const int64_t n = csr_entries(nnz_dev, cap);
  const int64_t e0 = t * kCsrTile, e1 = e0 + kCsrTile < n ? e0 + kCsrTile : n;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
    const int32_t r = rows[i];
    if (r >= 0 && r < n_node) atomicAdd(&s_h[r >> s1], 2u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[t * nb + b] = s_h[b];
}

template <typename V>
__global__ __launch_bounds__(256) void k_pass1_csr(const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
                                                 const V* __restrict__ vals, const V* __restrict__ res,
                                                 const int64_t* __restrict__ nnz_dev, int64_t cap, int64_t n_node,
                                                 int s1, int nb, const uint32_t* __restrict__ off1,
                                                 uint16_t* __restrict__ orow, uint32_t* __restrict__ ocol,
                                                 V* __restrict__ oval, uint32_t* __restrict__ emax) {
  constexpr int NT = 256, PER = kCsrTile / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const Pass1Smem<V, NT> sm(smem, 2 * kCsrTile, nb);
  const int64_t t = blockIdx.x;
  for (int b = threadIdx.x; b < nb; b += NT) {
    sm.cnt[b] = 0;
    sm.base[b] = off1[t * nb + b];
  }
  if (threadIdx.x == 0) *sm.emax = 0;
  __syncthreads();
  const int64_t n = csr_entries(nnz_dev, cap);
  const int64_t e0 = t * kCsrTile;
  int32_t r[PER];
  uint32_t q[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = e0 + u * NT + threadIdx.x;
    r[u] = i < n ? rows[i] : -1;
    if (r[u] >= n_node) r[u] = -1;
    if (r[u] >= 0) q[u] = atomicAdd(&sm.cnt[r[u] >> s1], 2u);
  }
  __syncthreads();
  const uint32_t n_items = block_scan_array(sm.cnt, nb, sm.scan);
  uint32_t em = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (r[u] < 0) continue;
    const int64_t i = e0 + u * NT + threadIdx.x;
    const uint32_t pos = sm.cnt[r[u] >> s1] + q[u];
    const uint64_t key = (uint64_t)(uint32_t)r[u] << 32 | (uint32_t)cols[i];
    const V h = vals[i];
    sm.key[pos] = key;
    sm.val[pos] = h;
    sm.key[pos + 1] = key;
    sm.val[pos + 1] = res[i];
    const uint32_t ep = (uint32_t)biased_exponent((double)h);  // |res| <= |h|
    em = (ep > em && ep < 0x7FF) ? ep : em;
  }
  if (em) atomicMax(sm.emax, em);
  __syncthreads();
  if (threadIdx.x == 0 && *sm.emax) atomicMax(emax, *sm.emax);
  pass1_write(sm, n_items, s1, NT, orow, ocol, oval);
}

// ------------------------------------------------------------------------ pass 2
// A bucket's pairs are cut into segments of SEG; segment ids run over all buckets
// (segbase[b] is the first segment of bucket b, segbase[nb] their number).

// seg2b[s] = bucket of segment s (one workgroup per bucket)
__global__ __launch_bounds__(256) void k_seg_map(const uint32_t* __restrict__ segbase, uint32_t* __restrict__ seg2b) {
  const uint32_t b = blockIdx.x;
  for (uint32_t s = segbase[b] + threadIdx.x; s < segbase[b + 1]; s += blockDim.x) seg2b[s] = b;
}

// histogram of sub-buckets ((row >> s2) mod p2) per segment: hist2[s * p2 + j]
// s[k] += 1 for each of N keys, one LDS atomic per run of equal consecutive keys (under a
// natural numbering neighbouring pairs mostly share a sub-bucket, and their increments
// would otherwise serialise on one address: 27M bricks, histogram 2.26 -> 1.01 ms)
template <int N>
__device__ __forceinline__ void count_runs(uint32_t* s, const uint32_t (&k)[N]) {
  uint32_t cur = k[0], run = 1;
#pragma unroll
  for (int i = 1; i < N; ++i) {
    if (k[i] == cur) {
      ++run;
    } else {
      atomicAdd(&s[cur], run);
      cur = k[i];
      run = 1;
    }
  }
  atomicAdd(&s[cur], run);
}

template <int SEG>
__global__ __launch_bounds__(256) void k_hist2(const uint16_t* __restrict__ irow, const uint32_t* __restrict__ bstart,
                                               const uint32_t* __restrict__ segbase,
                                               const uint32_t* __restrict__ seg2b, int nb, int s2, int p2,
                                               uint32_t* __restrict__ hist2) {
  extern __shared__ uint32_t s_h[];  // [p2]
  const uint32_t sid = blockIdx.x;
  if (sid >= segbase[nb]) return;
  const uint32_t b = seg2b[sid], s = sid - segbase[b];
  for (int j = threadIdx.x; j < p2; j += blockDim.x) s_h[j] = 0;
  __syncthreads();
  const uint32_t be = bstart[b + 1];
  const uint32_t i0 = bstart[b] + s * SEG, i1 = (i0 + SEG < be) ? i0 + SEG : be;
  const uint32_t mask = (uint32_t)p2 - 1;
  // eight row indices per 16-byte load over the 8-aligned middle of the range (irow is
  // 256-byte aligned); the ragged ends one by one
  const uint32_t a0 = (i0 + 7u) & ~7u, a1 = i1 & ~7u;
  if (a0 >= a1) {
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&s_h[(irow[i] >> s2) & mask], 1u);
  } else {
    for (uint32_t i = i0 + threadIdx.x; i < a0; i += blockDim.x) atomicAdd(&s_h[(irow[i] >> s2) & mask], 1u);
    for (uint32_t i = a1 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&s_h[(irow[i] >> s2) & mask], 1u);
    const uint4* __restrict__ w = (const uint4*)(irow + a0);
    for (uint32_t j = threadIdx.x; j < (a1 - a0) / 8; j += blockDim.x) {
      const uint4 v = w[j];
      const uint32_t k[8] = {((v.x & 0xFFFFu) >> s2) & mask, ((v.x >> 16) >> s2) & mask,
                             ((v.y & 0xFFFFu) >> s2) & mask, ((v.y >> 16) >> s2) & mask,
                             ((v.z & 0xFFFFu) >> s2) & mask, ((v.z >> 16) >> s2) & mask,
                             ((v.w & 0xFFFFu) >> s2) & mask, ((v.w >> 16) >> s2) & mask};
      count_runs<8>(s_h, k);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < p2; j += blockDim.x) hist2[(int64_t)sid * p2 + j] = s_h[j];
}

// One workgroup per bucket b: for each sub-bucket column j, the exclusive prefix of
// hist2 over the bucket's segments (in place), then the sub-bucket starts
// sbb[b * p2 + j] (sbb[nb * p2] = number of pairs).  A segment's run for sub-bucket j
// starts at sbb[b * p2 + j] + hist2[s * p2 + j].
__global__ __launch_bounds__(256) void k_colscan(uint32_t* __restrict__ hist2, const uint32_t* __restrict__ bstart,
                                                 const uint32_t* __restrict__ segbase, int nb, int p2,
                                                 uint32_t* __restrict__ sbb) {
  __shared__ uint32_t s_tot[1024];
  __shared__ uint32_t s_scan[8];
  const int b = blockIdx.x;
  const uint32_t sa = segbase[b], se = segbase[b + 1];
  for (int j = threadIdx.x; j < p2; j += blockDim.x) {
    uint32_t run = 0;
    uint32_t* col = hist2 + (int64_t)sa * p2 + j;
    uint32_t s = sa;
    for (; s + 8 <= se; s += 8, col += 8 * (int64_t)p2) {  // eight loads in flight
      uint32_t h[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) h[q] = col[q * (int64_t)p2];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        col[q * (int64_t)p2] = run;
        run += h[q];
      }
    }
    for (; s < se; ++s, col += p2) {
      const uint32_t h = *col;
      *col = run;
      run += h;
    }
    s_tot[j] = run;
  }
  __syncthreads();
  block_scan_array(s_tot, p2, s_scan);
  const uint32_t bs = bstart[b];
  for (int j = threadIdx.x; j < p2; j += blockDim.x) sbb[(int64_t)b * p2 + j] = bs + s_tot[j];
  if (b == nb - 1 && threadIdx.x == 0) sbb[(int64_t)nb * p2] = bstart[nb];
}

// scatter a segment into its sub-buckets; output key = row_local << colbits | col
template <typename V, int SEG, int NT>
__global__ __launch_bounds__(NT) void k_scatter2(const uint16_t* __restrict__ irow, const uint32_t* __restrict__ icol,
                                                  const V* __restrict__ ival, const uint32_t* __restrict__ bstart,
                                                  const uint32_t* __restrict__ segbase,
                                                  const uint32_t* __restrict__ seg2b,
                                                  const uint32_t* __restrict__ off2, const uint32_t* __restrict__ sbb,
                                                  int nb, int s2, int p2, int colbits, uint32_t* __restrict__ okey,
                                                  V* __restrict__ oval) {
  extern __shared__ __align__(16) unsigned char smem[];
  V* s_val = (V*)smem;                          // [SEG]
  uint32_t* s_key = (uint32_t*)(s_val + SEG);   // [SEG]
  uint16_t* s_sb = (uint16_t*)(s_key + SEG);    // [SEG] sub-bucket of staged pair
  uint32_t* s_cnt = (uint32_t*)(s_sb + SEG);    // [p2] pairs per sub-bucket, then local starts
  uint32_t* s_off = s_cnt + p2;                 // [p2] global offsets
  uint32_t* s_scan = s_off + p2;                // [NT/64 + 1]
  const uint32_t sid = (uint32_t)xcd_item(blockIdx.x, gridDim.x);
  if (sid >= segbase[nb]) return;
  const uint32_t b = seg2b[sid], s = sid - segbase[b];
  for (int j = threadIdx.x; j < p2; j += blockDim.x) {
    s_cnt[j] = 0;
    s_off[j] = sbb[(int64_t)b * p2 + j] + off2[(int64_t)sid * p2 + j];
  }
  __syncthreads();
  const uint32_t be = bstart[b + 1];
  const uint32_t i0 = bstart[b] + s * SEG, i1 = (i0 + SEG < be) ? i0 + SEG : be;
  const uint32_t mask = (uint32_t)p2 - 1, rmask = (1u << s2) - 1;
  constexpr int PER = SEG / NT;
  uint32_t rr[PER], cc[PER], rk[PER];
  V vv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {  // every load issued first (indices clamped into the segment)
    const uint32_t i = i0 + q * NT + threadIdx.x;
    const uint32_t ic = i < i1 ? i : i0;
    rr[q] = irow[ic];
    cc[q] = icol[ic];
    vv[q] = ival[ic];
  }
  // rank of each pair within its sub-bucket, then the local run starts
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = i0 + q * NT + threadIdx.x;
    if (i < i1) rk[q] = atomicAdd(&s_cnt[(rr[q] >> s2) & mask], 1u);
  }
  __syncthreads();
  block_scan_array(s_cnt, p2, s_scan);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = i0 + q * NT + threadIdx.x;
    if (i < i1) {
      const uint32_t j = (rr[q] >> s2) & mask;
      const uint32_t pos = s_cnt[j] + rk[q];
      s_key[pos] = ((rr[q] & rmask) << colbits) | cc[q];
      s_val[pos] = vv[q];
      s_sb[pos] = (uint16_t)j;
    }
  }
  __syncthreads();
  const uint32_t n = i1 - i0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t j = s_sb[i];
    const uint32_t g = s_off[j] + (i - s_cnt[j]);
    okey[g] = s_key[i];
    oval[g] = s_val[i];
  }
}

// The first kHeavyPar heavy sub-buckets of the list are split, and their first-level
// digit ranges reduced, by many workgroups (k_heavy_rows, k_heavy_layout, k_heavy_hist,
// k_heavy_starts, k_heavy_scatter, k_pass3_heavy_ranges); k_pass3_heavy_finish then
// sums up each one's entries and k_final_heavy gathers them from the ranges.
// k_pass3_heavy clears their tables and takes the other listed sub-buckets whole.
// The first-level digits follow the rows: row r of a sub-bucket gets n_r digits (a
// power of two, none for a row without pairs), each covering 2^(colbits) / n_r columns,
// with n_r about kHvyShare times the row's share of the pairs, at most one digit per
// leaf width of columns, and at least 2^(colbits - 23) so that a digit is at most 2^23
// keys wide (split once more into leaves).  A row holding most pairs of its sub-bucket
// thus gets 2048 digits, leaf-wide up to 2^23 columns, which many workgroups reduce
// side by side.  The digits of all rows total at most kHvyShare + 256 + 256 =
// kHvyDigits.
constexpr int kHeavyPar = 64;
constexpr int kHvyDigits = 4096;  // first-level digits at most
constexpr uint32_t kHvyShare = 3584;
constexpr int kHvyRows = 256;  // rows of a sub-bucket at most
constexpr int kHvyWords = (kHvyDigits + 1) + kHvyDigits + 3 * kHvyRows + (kHvyRows + 1) + 4;
struct HeavyTable {
  uint32_t* st;     // [kHvyDigits + 1] digit starts (absolute pair positions)
  uint32_t* hist;   // [kHvyDigits] pairs of each digit, then the scatter's cursors
  uint32_t* ucnt;   // the same words once the scatter is done: the entries of each digit
                    // range (every range writes its own), then their offsets
  uint32_t* rcnt;   // [kHvyRows] entries of each row
  uint32_t* rpair;  // [kHvyRows] pairs of each row
  uint32_t* rsh;    // [kHvyRows] column shift of each row's digits
  uint32_t* rbase;  // [kHvyRows + 1] first digit of each row; rbase[kHvyRows] = digits
  uint32_t* meta;   // [4] digits
  __device__ HeavyTable(uint32_t* hvy, uint32_t it) {
    st = hvy + (size_t)it * kHvyWords;
    hist = st + kHvyDigits + 1;
    ucnt = hist;
    rcnt = hist + kHvyDigits;
    rpair = rcnt + kHvyRows;
    rsh = rpair + kHvyRows;
    rbase = rsh + kHvyRows;
    meta = rbase + kHvyRows + 1;
  }
};

// table entry it of a listed sub-bucket: the row counts cleared
__device__ __forceinline__ void heavy_table_init(uint32_t* hvy, uint32_t it) {
  const HeavyTable t(hvy, it);
  for (uint32_t r = threadIdx.x; r < (uint32_t)kHvyRows; r += blockDim.x) {
    t.rcnt[r] = 0u;
    t.rpair[r] = 0u;
  }
}

// first-level digit of key k (row k >> colbits) from the layout in LDS
__device__ __forceinline__ uint32_t heavy_digit(uint32_t k, int colbits, const uint32_t* s_rbase,
                                                const uint32_t* s_rsh) {
  const uint32_t r = k >> colbits;
  return s_rbase[r] + ((k & ((1u << colbits) - 1u)) >> s_rsh[r]);
}

// ------------------------------------------------------------------------ pass 3
// home slot of a packed key in a table of HT (a power of two) slots: the top bits of
// the key mixed by xor-shift, multiply by 2^32/phi, xor-shift.  A plain multiplicative
// hash lets the row bits (the key's top bits) and the columns of a naturally numbered
// grid interfere: on the 300^3 brick box it gave 1.9 probes per insert on average and
// runs of up to 15, against 1.1 and 4 for the mixed key (the reduce 1.9x slower)
template <int HT>
__device__ __forceinline__ uint32_t slot_hash(uint32_t k) {
  constexpr int bits = __builtin_ctz(HT);
  k ^= k >> 15;
  k *= 0x9E3779B1u;
  k ^= k >> 13;
  return k >> (32 - bits);
}

// One workgroup per sub-bucket g (rows [g << s2, ...)).  Writes its unique entries in
// CSR order to tcol/tval[sbb[g] + f], each row's first entry (relative to the
// sub-bucket) to rowoff, its total to usub[g].  A sub-bucket of more than 2^16 pairs
// or more distinct entries than the table holds is appended to ov_list (count in
// *ov_count) and left to k_pass3_heavy.
// Sub-buckets run in their natural order: under a random numbering the lower-triangle
// pairs of a row grow with its id, so an even interleave keeps the XCDs balanced.
// With RES, each entry's residual (the exact sum minus its rounding) goes to tres too.
template <typename V, int HT, bool RES = false>
__global__ __launch_bounds__(256) void k_pass3(uint32_t* __restrict__ ikey, V* __restrict__ ival,
                                               const uint32_t* __restrict__ sbb, int s2, int colbits, int64_t n_node,
                                               const uint32_t* __restrict__ emax, int32_t* __restrict__ tcol,
                                               V* __restrict__ tval, V* __restrict__ tres,
                                               uint32_t* __restrict__ rowoff, uint32_t* __restrict__ usub,
                                               uint32_t* __restrict__ ov_list, uint32_t* __restrict__ ov_count) {
  constexpr int NT = 256, PER = 8;
  // once summed, each slot's value (and residual) is kept in place of its low chunk sum,
  // which frees the high chunk sums for the columns grouped by row (one array fewer); a
  // double with its double residual needs both words.  The per-row arrays are sized by
  // the sub-bucket's rows at launch and the columns are grouped by row through cursors
  // (no per-slot index within the row): 22.4 KB at 1024 slots, seven workgroups per CU
  constexpr bool kSepCols = RES && sizeof(V) == 8;
  __shared__ uint32_t s_key[HT];
  __shared__ unsigned long long s_lo[HT];  // sum of low 48-bit chunks, then value (+ residual)
  __shared__ unsigned long long s_hi[HT];  // sum of signed high chunks, then the columns
  __shared__ uint16_t s_slot[HT];  // occupied slots, in insertion order
  __shared__ uint32_t s_sep[kSepCols ? HT : 1];
  __shared__ uint32_t s_over, s_nu;
  extern __shared__ uint32_t s_rows[];  // 3 << s2 words: entries per row, row offsets, cursors
  uint32_t* const s_rc = s_rows;
  uint32_t* const s_ro = s_rows + (1 << s2);
  uint32_t* const s_cur = s_rows + (2 << s2);
  uint32_t* const s_lcol = kSepCols ? s_sep : (uint32_t*)s_hi;  // columns of the slots, grouped by row

  const int64_t g = blockIdx.x;
  const uint32_t beg = sbb[g], end = sbb[g + 1];
  const int64_t r0 = g << s2;
  const int64_t rr = n_node - r0;
  const int R = rr <= 0 ? 0 : (rr < ((int64_t)1 << s2) ? (int)rr : (1 << s2));
  const int F = 1117 - (int)*emax;
  const uint32_t cmask = (1u << colbits) - 1;

  for (int h = threadIdx.x; h < HT; h += NT) {
    s_key[h] = kEmptyKey;
    s_lo[h] = 0ull;
    s_hi[h] = 0ull;
  }
  for (int r = threadIdx.x; r < (1 << s2); r += NT) s_rc[r] = 0;
  // more than 2^16 pairs could overflow the chunk sums: left to the heavy kernel
  if (threadIdx.x == 0) {
    s_over = (end - beg > (1u << 16)) ? 1u : 0u;
    s_nu = 0;
  }
  __syncthreads();
  // stream the pairs into the table: PER loads per lane in flight (indices clamped into
  // the range; the empty asm keeps the compiler from sinking a load into the branch
  // that first uses it)
  if (!s_over) {
    // (offsets from the sub-bucket's first pair: below 2^16 here)
    const uint32_t n = end - beg;
    const uint32_t* const kp = ikey + beg;
    const V* const vp = ival + beg;
    for (uint32_t j0 = 0; j0 < n; j0 += PER * NT) {
      uint32_t kk[PER];
      V vv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const uint32_t j = j0 + u * NT + threadIdx.x;
        const uint32_t jc = (j < n ? j : 0u) & 0xffffu;
        kk[u] = kp[jc];
        vv[u] = vp[jc];
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) asm volatile("" : "+v"(kk[u]), "+v"(vv[u]));
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (j0 + u * NT + threadIdx.x >= n) continue;
        const uint32_t key = kk[u];
        // one compare-and-swap per probe: it returns the empty marker when this lane
        // took the slot, the key when the entry was there already, else another key
        uint32_t h = slot_hash<HT>(key);
        uint32_t k = atomicCAS(&s_key[h], kEmptyKey, key);
        int probes = 0;
#pragma unroll 1
        while (k != kEmptyKey && k != key && ++probes < HT) {
          h = (h + 1) & (HT - 1);
          k = atomicCAS(&s_key[h], kEmptyKey, key);
        }
        if (k != kEmptyKey && k != key) {  // the table is full
          s_over = 1;
          continue;
        }
        uint64_t c0;
        int64_t c1;
        to_chunks(vv[u], F, c0, c1);
        atomicAdd(&s_lo[h], (unsigned long long)c0);
        atomicAdd(&s_hi[h], (unsigned long long)c1);
      }
    }
  }
  __syncthreads();
  if (s_over) {  // left to k_pass3_heavy
    if (threadIdx.x == 0) ov_list[atomicAdd(ov_count, 1u)] = (uint32_t)g;
    return;
  }
  // list the occupied slots and count the entries of each row (once per entry here
  // rather than on the insertion path of every pair)
  for (int h = threadIdx.x; h < HT; h += NT) {
    const uint32_t k = s_key[h];
    if (k != kEmptyKey) {
      s_slot[atomicAdd(&s_nu, 1u)] = (uint16_t)h;
      atomicAdd(&s_rc[k >> colbits], 1u);
    }
  }
  __syncthreads();
  // order the U entries by (row, col): the row counts scanned by one
  // wave while the others round each sum to its value, the entries grouped by row, then
  // ranked by column within their row
  const uint32_t U = s_nu;
  const int RB = 1 << s2;  // rows of a full sub-bucket (<= 256)
  for (uint32_t f = threadIdx.x < 64 ? U : threadIdx.x - 64; f < U; f += NT - 64) {
    const uint32_t h = s_slot[f];
    uint64_t lo, hi;
    join48(s_lo[h], (int64_t)s_hi[h], lo, hi);
    const V hv = from_fixed_as<V>(lo, hi, F);
    if constexpr (sizeof(V) == 8) {
      s_lo[h] = (unsigned long long)__double_as_longlong((double)hv);
      if constexpr (RES) s_hi[h] = (unsigned long long)__double_as_longlong((double)fixed_residual<V>(lo, hi, F, hv));
    } else {
      const uint32_t rv = RES ? __float_as_uint((float)fixed_residual<V>(lo, hi, F, hv)) : 0u;
      s_lo[h] = ((unsigned long long)rv << 32) | __float_as_uint((float)hv);
    }
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = lane * 4 + k;
      v[k] = r < RB ? s_rc[r] : 0u;
      sum += v[k];
    }
    uint32_t x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    uint32_t run = x - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = lane * 4 + k;
      if (r < RB) {
        s_ro[r] = run;
        s_cur[r] = run;
      }
      run += v[k];
    }
  }
  __syncthreads();
  for (uint32_t f = threadIdx.x; f < U; f += NT) {
    const uint32_t h = s_slot[f];
    const uint32_t k = s_key[h];
    s_lcol[atomicAdd(&s_cur[k >> colbits], 1u)] = k & cmask;
  }
  __syncthreads();
  for (uint32_t f = threadIdx.x; f < U; f += NT) {
    const uint32_t h = s_slot[f];
    const uint32_t k = s_key[h];
    const uint32_t row = k >> colbits, col = k & cmask;
    const uint32_t ro = s_ro[row], nr = s_rc[row];
    uint32_t rank = 0;
    for (uint32_t q = 0; q < nr; ++q) rank += (s_lcol[ro + q] < col) ? 1u : 0u;
    const uint32_t pos = ro + rank;
    tcol[beg + pos] = (int32_t)col;
    const unsigned long long w = s_lo[h];
    if constexpr (sizeof(V) == 8) {
      tval[beg + pos] = (V)__longlong_as_double((long long)w);
      if constexpr (RES) tres[beg + pos] = (V)__longlong_as_double((long long)s_hi[h]);
    } else {
      tval[beg + pos] = (V)__uint_as_float((uint32_t)w);
      if constexpr (RES) tres[beg + pos] = (V)__uint_as_float((uint32_t)(w >> 32));
    }
  }
  for (int r = threadIdx.x; r < R; r += NT) rowoff[r0 + r] = s_ro[r];
  if (threadIdx.x == 0) usub[g] = U;
}

// ------------------------------------------------------------ heavy sub-buckets
// A sub-bucket that overflows pass 3 (a node shared by very many elements: its row holds
// more distinct entries than an LDS table, or more than 2^16 pairs) is split by key into
// ranges of at most kLeafKeys keys, each summed into a direct-addressed LDS table.  The
// first kHeavyPar listed are split by the whole device (k_heavy_*, the tables above);
// each further one is reduced whole by one 1024-lane workgroup of k_pass3_heavy:
//   - the key range [kmin, kmax] of the sub-bucket; a range wider than kLeafKeys is split
//     into at most 2048 digit ranges of 2^shift keys (a histogram, its scan and a
//     scatter into the other buffer, at the same place), twice at most for 31-bit keys;
//   - each leaf range (in key order) sums its pairs into a direct-addressed LDS table,
//     one slot per key, with the exact chunk sums of pass 3, carried into a third word
//     after every 2^16 pairs (so any number of pairs sums exactly); then the occupied
//     slots, in slot order = (row, col) order, are written after the entries before.
// Output as pass 3.  The pairs alternate between (ikey, ival) and (akey, aval), the
// pass-1 arrays, which also receive the output (tcol / tval): a leaf writes at most as
// many entries as it has pairs, so the output never reaches a pair not yet read.
constexpr int kLeafKeys = 4096, kHeavyThreads = 1024, kDigits = 2048;

struct HeavySmem {
  unsigned long long* lo;  // [kLeafKeys] sum of low 48-bit chunks
  long long* hi;           // [kLeafKeys] sum of signed high chunks (bits 48..)
  long long* top;          // [kLeafKeys] carries above bit 96
  uint8_t* occ;            // [kLeafKeys] 1 for an occupied slot (byte stores: no atomics)
  uint32_t* hist;          // [kDigits] digit counts, then cursors
  uint32_t* start;         // [2][kDigits + 1] digit starts of the two split levels
  uint32_t* rowcnt;        // [256] entries per row of the sub-bucket
  uint32_t* scan;          // [kHeavyThreads / 64 + 1]
  uint32_t* misc;          // [4]
  __device__ explicit HeavySmem(unsigned char* p) {
    lo = (unsigned long long*)p;
    hi = (long long*)(lo + kLeafKeys);
    top = hi + kLeafKeys;
    occ = (uint8_t*)(top + kLeafKeys);
    hist = (uint32_t*)(occ + kLeafKeys);
    start = hist + kDigits;
    rowcnt = start + 2 * (kDigits + 1);
    scan = rowcnt + 256;
    misc = scan + kHeavyThreads / 64 + 1;
  }
  static constexpr size_t bytes() {
    return (size_t)kLeafKeys * 25 + 4 * ((size_t)kDigits + 2 * (kDigits + 1) + 256 + kHeavyThreads / 64 + 1 + 4);
  }
};

// block-wide barrier after global stores that other waves of the workgroup read next:
// the barrier's workgroup-scope fence waits for the stores, and the waves of one
// workgroup share the compute unit's write-through vector cache (an agent-scope fence
// here would write back and invalidate the whole L2 at every call)
__device__ __forceinline__ void heavy_sync() { __syncthreads(); }

// Stream [a, b) of (key, value) pairs through f(key, value, ok), kHeavyPer pairs per lane
// in flight (indices clamped into the range; the empty asm keeps the loads ahead of the
// atomics that use them).  f is called by every lane in uniform control flow, ok telling
// whether its pair is in the range, so that f can combine the lanes of a wave.
// WITH_VAL = false reads the keys only.
constexpr int kHeavyPer = 8;
template <bool WITH_VAL, typename V, typename Fn>
__device__ __forceinline__ void heavy_stream(const uint32_t* key, const V* val, uint32_t a, uint32_t b, Fn f) {
  for (uint32_t i0 = a; i0 < b; i0 += kHeavyPer * kHeavyThreads) {
    uint32_t kk[kHeavyPer];
    V vv[kHeavyPer] = {};
#pragma unroll
    for (int u = 0; u < kHeavyPer; ++u) {
      const uint32_t i = i0 + u * kHeavyThreads + threadIdx.x;
      const uint32_t ic = i < b ? i : a;
      kk[u] = key[ic];
      if constexpr (WITH_VAL) vv[u] = val[ic];
    }
#pragma unroll
    for (int u = 0; u < kHeavyPer; ++u) {
      if constexpr (WITH_VAL)
        asm volatile("" : "+v"(kk[u]), "+v"(vv[u]));
      else
        asm volatile("" : "+v"(kk[u]));
    }
#pragma unroll
    for (int u = 0; u < kHeavyPer; ++u) f(kk[u], vv[u], i0 + u * kHeavyThreads + threadIdx.x < b);
  }
}

// A heavy node's diagonal (or one column of its row) can own most pairs of a range, and
// atomics on one LDS address serialise.  Each wave therefore takes its first lane's
// digit or slot as "hot": when more than one lane holds it, those lanes are combined into
// one atomic by the first lane (heavy_hot returns their mask, else 0).
__device__ __forceinline__ uint64_t heavy_hot(uint32_t x, bool ok, uint32_t& hot) {
  hot = __builtin_amdgcn_readfirstlane(x);
  const uint64_t m = __ballot(ok && x == hot);
  return __popcll(m) > 1 ? m : 0ull;
}

template <typename V>
__device__ void heavy_split(const HeavySmem& sm, const uint32_t* skey, const V* sval, uint32_t* dkey, V* dval,
                            uint32_t a, uint32_t b, uint32_t kmin, int shift, int nd, uint32_t* st) {
  const int lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < nd; d += kHeavyThreads) sm.hist[d] = 0;
  __syncthreads();
  heavy_stream<false>(skey, sval, a, b, [&](uint32_t k, V, bool ok) {
    const uint32_t d = (k - kmin) >> shift;
    uint32_t hot;
    const uint64_t m = heavy_hot(d, ok, hot);
    if (ok && !((m >> lane) & 1ull)) atomicAdd(&sm.hist[d], 1u);
    if (lane == 0 && m) atomicAdd(&sm.hist[hot], (uint32_t)__popcll(m));
  });
  __syncthreads();
  block_scan_array(sm.hist, nd, sm.scan);  // (ends with a barrier)
  for (int d = threadIdx.x; d < nd; d += kHeavyThreads) st[d] = a + sm.hist[d];
  if (threadIdx.x == 0) st[nd] = b;
  __syncthreads();
  heavy_stream<true>(skey, sval, a, b, [&](uint32_t k, V v, bool ok) {
    const uint32_t d = (k - kmin) >> shift;
    uint32_t hot;
    const uint64_t m = heavy_hot(d, ok, hot);
    uint32_t base = 0;
    if (lane == 0 && m) base = atomicAdd(&sm.hist[hot], (uint32_t)__popcll(m));
    base = __shfl(base, 0, 64);
    const bool mine = (m >> lane) & 1ull;
    uint32_t pos = 0;
    if (mine)
      pos = a + base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
    else if (ok)
      pos = a + atomicAdd(&sm.hist[d], 1u);
    if (ok) {
      dkey[pos] = k;
      dval[pos] = v;
    }
  });
  heavy_sync();
}

// carry the low and high chunk sums of the occupied slots upward: lo < 2^48, hi < 2^48
__device__ __forceinline__ void heavy_normalise(const HeavySmem& sm) {
  constexpr unsigned long long M48 = (1ull << 48) - 1;
  for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
    if (!sm.occ[h]) continue;
    const unsigned long long l = sm.lo[h];
    const long long x = sm.hi[h] + (long long)(l >> 48);
    sm.lo[h] = l & M48;
    sm.top[h] += x >> 48;  // arithmetic shift: floor division
    sm.hi[h] = (long long)((unsigned long long)x & M48);
  }
}

// pairs per round of a leaf: the carried sums (below 2^48) plus kRound chunks (below
// 2^48 unsigned, below 2^47 in magnitude signed) stay inside 64 bits
constexpr uint32_t kRound = 65532;

// the exact sums of the leaf's pairs [a, b) (keys in [kmin, kmin + kLeafKeys)) into the
// LDS slots, carried after every round (lo, hi below 2^48; occ set)
template <typename V>
__device__ void heavy_leaf_sum(const HeavySmem& sm, const uint32_t* key, const V* val, uint32_t a, uint32_t b,
                               uint32_t kmin, int F) {
  const int lane = threadIdx.x & 63;
  // the wave's kept slot: once a slot has been hot (held by more than one lane), the
  // lanes that meet it again while it is the wave's first lane's slot add its chunks to
  // their own sums, which are summed over the wave and added once, at the end of the
  // round (a key that owns most of the leaf, such as a heavy node's diagonal, then costs
  // two register additions per pair)
  for (uint32_t r = a; r < b; r += kRound) {
    const uint32_t re = b - r > kRound ? r + kRound : b;
    uint32_t kept = kEmptyKey;  // (uniform)
    unsigned long long k0 = 0ull;
    long long k1 = 0ll;
    const auto flush = [&]() {  // the kept sums over the wave, added to the kept slot
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        k0 += __shfl_xor(k0, o, 64);
        k1 += __shfl_xor(k1, o, 64);
      }
      if (lane == 0) {
        atomicAdd(&sm.lo[kept], k0);
        atomicAdd((unsigned long long*)&sm.hi[kept], (unsigned long long)k1);
        sm.occ[kept] = 1;
      }
      k0 = 0ull;
      k1 = 0ll;
    };
    heavy_stream<true>(key, val, r, re, [&](uint32_t k, V v, bool ok) {
      const uint32_t h = k - kmin;
      uint64_t c0;
      int64_t c1;
      to_chunks(v, F, c0, c1);
      uint32_t hot;
      const uint64_t m = heavy_hot(h, ok, hot);
      const bool mine = (m >> lane) & 1ull;
      if (ok && !mine) {
        atomicAdd(&sm.lo[h], (unsigned long long)c0);
        atomicAdd((unsigned long long*)&sm.hi[h], (unsigned long long)c1);
        sm.occ[h] = 1;
      }
      if (m) {
        if (hot != kept) {  // (uniform) a new kept slot: the old one's sums go first
          if (kept != kEmptyKey) flush();
          kept = hot;
        }
        if (mine) {  // (64 lanes x 64 pairs of a round: the sums stay below 2^60)
          k0 += c0;
          k1 += c1;
        }
      }
    });
    if (kept != kEmptyKey) flush();
    __syncthreads();
    heavy_normalise(sm);
    __syncthreads();
  }
}

// the occupied LDS slots (carried sums) as entries, appended in key order at tcol /
// tval [u0 ...), the slots cleared; returns the number of entries
template <typename V, bool RES>
__device__ uint32_t heavy_leaf_emit(const HeavySmem& sm, uint32_t kmin, int F, int colbits, int32_t* tcol, V* tval,
                                    V* tres, uint32_t u0) {
  const int lane = threadIdx.x & 63;
  // the occupied slots in order: kLeafKeys / kHeavyThreads consecutive slots per lane
  constexpr int PL = kLeafKeys / kHeavyThreads;
  const int h0 = threadIdx.x * PL;
  static_assert(PL == 4, "four slot flags per lane are read as one word");
  const uint32_t fw = *(const uint32_t*)(sm.occ + h0);  // byte j: slot h0 + j
  const uint32_t bits = (fw & 1u) | ((fw >> 7) & 2u) | ((fw >> 14) & 4u) | ((fw >> 21) & 8u);
  uint32_t total;
  uint32_t pos = u0 + block_scan_u32(__popc(bits), sm.scan, &total);
  const uint32_t cmask = (1u << colbits) - 1;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const bool occ = (bits >> j) & 1u;
    const int h = h0 + j;
    const uint32_t k = kmin + (uint32_t)h;
    // entries per row: a range spans few rows, so the lanes of a wave mostly share one
    uint32_t hot;
    const uint64_t m = heavy_hot(k >> colbits, occ, hot);
    if (occ && !((m >> lane) & 1ull)) atomicAdd(&sm.rowcnt[k >> colbits], 1u);
    if (lane == 0 && m) atomicAdd(&sm.rowcnt[hot], (uint32_t)__popcll(m));
    if (!occ) continue;
    // value = lo + hi 2^48 + top 2^96, lo and hi in [0, 2^48): as a 128-bit integer
    const unsigned long long l = sm.lo[h], x = (unsigned long long)sm.hi[h];
    const long long t = sm.top[h];
    const uint64_t qlo = l | (x << 48);
    const uint64_t qhi = (x >> 16) | ((uint64_t)t << 32);
    const V hv = from_fixed_as<V>(qlo, qhi, F);
    tcol[pos] = (int32_t)(k & cmask);
    tval[pos] = hv;
    if constexpr (RES) tres[pos] = fixed_residual<V>(qlo, qhi, F, hv);
    sm.lo[h] = 0ull;
    sm.hi[h] = 0ll;
    sm.top[h] = 0ll;
    ++pos;
  }
  __syncthreads();
  if (threadIdx.x < kLeafKeys / 4) ((uint32_t*)sm.occ)[threadIdx.x] = 0u;
  heavy_sync();
  return total;
}

// sums of the leaf's pairs [a, b) (keys in [kmin, kmin + kLeafKeys)), appended in key
// order at tcol / tval [u0 ...); returns the number of entries
template <typename V, bool RES>
__device__ uint32_t heavy_leaf(const HeavySmem& sm, const uint32_t* key, const V* val, uint32_t a, uint32_t b,
                               uint32_t kmin, int F, int colbits, int32_t* tcol, V* tval, V* tres, uint32_t u0) {
  heavy_leaf_sum<V>(sm, key, val, a, b, kmin, F);
  return heavy_leaf_emit<V, RES>(sm, kmin, F, colbits, tcol, tval, tres, u0);
}

// Leaves of the split sub-buckets (first-level digit ranges no wider than a leaf) with
// more than kBigLeafPairs pairs, such as the one holding a heavy node's diagonal, are
// summed by several workgroups: k_heavy_starts lists up to kBigLeaves of them, each
// workgroup of k_heavy_bigleaf sums one round (kRound pairs) of one of them into its LDS
// slots and adds the carried sums (lo, hi below 2^48, top) of its occupied slots into
// the leaf's accumulator with 64-bit atomics (exact: a leaf of fewer than 2^31 pairs has
// fewer than 2^16 rounds), and k_pass3_heavy_ranges carries the accumulated sums once
// more and writes the leaf's entries.  Leaves beyond the list are summed as the others.
constexpr int kBigLeaves = 8;
constexpr uint32_t kBigLeafPairs = 2 * kRound;
constexpr int kBigRec = 8;  // words per listed leaf: it, d0, a, b, k0
constexpr int kBigListWords = 8 + kBigRec * kBigLeaves;
constexpr int kBigAccWords = 7 * kLeafKeys;  // lo, hi, top (64-bit) and occ (32-bit) per slot
constexpr size_t kBigWords = kBigListWords + (size_t)kBigLeaves * kBigAccWords;
struct BigLeaves {
  uint32_t* list;  // [0] leaves listed (may exceed kBigLeaves), then the records
  __device__ explicit BigLeaves(uint32_t* hvy) : list(hvy + (size_t)kHeavyPar * kHvyWords) {}
  __device__ uint32_t count() const { return list[0] < (uint32_t)kBigLeaves ? list[0] : (uint32_t)kBigLeaves; }
  __device__ uint32_t* rec(uint32_t i) const { return list + 8 + kBigRec * i; }
  __device__ unsigned long long* lo(uint32_t i) const {
    return (unsigned long long*)(list + kBigListWords + (size_t)i * kBigAccWords);
  }
  __device__ unsigned long long* hi(uint32_t i) const { return lo(i) + kLeafKeys; }
  __device__ unsigned long long* top(uint32_t i) const { return lo(i) + 2 * kLeafKeys; }
  __device__ uint32_t* occ(uint32_t i) const { return (uint32_t*)(lo(i) + 3 * kLeafKeys); }
};
static_assert(((size_t)kHeavyPar * kHvyWords + kBigListWords) % 2 == 0, "the accumulators are 8-byte aligned");

// split width for a key range of w keys: 0 for a leaf, else the digit shift
__device__ __forceinline__ int heavy_shift(uint32_t w) {
  if (w <= (uint32_t)kLeafKeys) return 0;
  const int bits = 32 - __clz(w - 1);  // keys need `bits` bits
  return bits - 11 > 12 ? bits - 11 : 12;  // at most kDigits digits
}

// One first-level digit range [a, b) of a heavy sub-bucket, in (akey, aval), keys in
// [k0, k0 + w): a leaf, or split again into (ikey, ival) at the same place and its leaves
// summed in key order.  Entries written from tcol / tval / tres [u0 ...); returns their
// number.  The range's pairs are all read before any entry is written, and a range has
// at most as many entries as pairs.
template <typename V, bool RES>
__device__ uint32_t heavy_range(const HeavySmem& sm, uint32_t* ikey, V* ival, uint32_t* akey, V* aval, uint32_t a,
                                uint32_t b, uint32_t k0, uint32_t w, int F, int colbits, int32_t* tcol, V* tval,
                                V* tres, uint32_t u0) {
  const int sh1 = heavy_shift(w);
  if (sh1 == 0) return heavy_leaf<V, RES>(sm, akey, aval, a, b, k0, F, colbits, tcol, tval, tres, u0);
  const int nd1 = (int)((w - 1) >> sh1) + 1;
  uint32_t* st1 = sm.start + (kDigits + 1);
  heavy_split<V>(sm, akey, aval, ikey, ival, a, b, k0, sh1, nd1, st1);
  uint32_t U = 0;
  for (int d1 = 0; d1 < nd1; ++d1) {  // leaves (sh1 = 12 after a first split)
    const uint32_t a1 = st1[d1], b1 = st1[d1 + 1];
    if (a1 == b1) continue;
    U += heavy_leaf<V, RES>(sm, ikey, ival, a1, b1, k0 + ((uint32_t)d1 << sh1), F, colbits, tcol, tval, tres, u0 + U);
  }
  return U;
}

// The listed sub-buckets after the first kHeavyPar, one workgroup each; its first
// kHeavyPar workgroups also clear the first kHeavyPar tables and the big-leaf count
// (the pair buffers alias the output, so they carry no __restrict__)
template <typename V, bool RES = false>
__global__ __launch_bounds__(kHeavyThreads) void k_pass3_heavy(uint32_t* ikey, V* ival, uint32_t* akey, V* aval,
                                                             const uint32_t* __restrict__ sbb, int s2, int colbits,
                                                             int64_t n_node, const uint32_t* __restrict__ emax,
                                                             V* __restrict__ tres, uint32_t* __restrict__ rowoff,
                                                             uint32_t* __restrict__ usub,
                                                             const uint32_t* __restrict__ ov_list,
                                                             const uint32_t* __restrict__ ov_count,
                                                             uint32_t* __restrict__ hvy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const HeavySmem sm(smem);
  const uint32_t n_over = *ov_count;
  // (launched with at least kHeavyPar workgroups)
  if (blockIdx.x < n_over && blockIdx.x < (uint32_t)kHeavyPar) heavy_table_init(hvy, blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0 && n_over) BigLeaves(hvy).list[0] = 0u;
  if ((uint32_t)kHeavyPar + blockIdx.x >= n_over) return;
  for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
    sm.lo[h] = 0ull;
    sm.hi[h] = 0ll;
    sm.top[h] = 0ll;
  }
  if (threadIdx.x < kLeafKeys / 4) ((uint32_t*)sm.occ)[threadIdx.x] = 0u;
  const int F = 1117 - (int)*emax;
  int32_t* const tcol = (int32_t*)akey;
  for (uint32_t it = (uint32_t)kHeavyPar + blockIdx.x; it < n_over; it += gridDim.x) {
    const int64_t g = ov_list[it];
    const uint32_t beg = sbb[g], end = sbb[g + 1];
    const int64_t r0 = g << s2;
    const int R = (int)min((int64_t)1 << s2, n_node - r0);
    for (int r = threadIdx.x; r < 256; r += kHeavyThreads) sm.rowcnt[r] = 0u;
    // key range
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    heavy_stream<false>(ikey, ival, beg, end, [&](uint32_t k, V, bool ok) {
      mn = ok && k < mn ? k : mn;
      mx = ok && k > mx ? k : mx;
    });
    if (threadIdx.x < 2) sm.misc[threadIdx.x] = threadIdx.x == 0 ? 0xFFFFFFFFu : 0u;
    __syncthreads();
    atomicMin(&sm.misc[0], mn);
    atomicMax(&sm.misc[1], mx);
    __syncthreads();
    const uint32_t kmin = sm.misc[0], w0 = sm.misc[1] - kmin + 1;
    __syncthreads();
    uint32_t U = 0;
    const int sh0 = heavy_shift(w0);
    if (sh0 == 0) {
      U = heavy_leaf<V, RES>(sm, ikey, ival, beg, end, kmin, F, colbits, tcol + beg, aval + beg,
                             RES ? tres + beg : nullptr, 0);
    } else {
      const int nd0 = (int)((w0 - 1) >> sh0) + 1;
      uint32_t* st0 = sm.start;
      heavy_split<V>(sm, ikey, ival, akey, aval, beg, end, kmin, sh0, nd0, st0);
      for (int d0 = 0; d0 < nd0; ++d0) {
        const uint32_t a = st0[d0], b = st0[d0 + 1];
        if (a == b) continue;
        const uint32_t k0 = kmin + ((uint32_t)d0 << sh0);
        const uint32_t w1 = (1u << sh0) < (kmin + w0 - k0) ? (1u << sh0) : (kmin + w0 - k0);
        U += heavy_range<V, RES>(sm, ikey, ival, akey, aval, a, b, k0, w1, F, colbits, tcol + beg, aval + beg,
                                 RES ? tres + beg : nullptr, U);
      }
    }
    // row offsets within the sub-bucket
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      uint32_t v[4], sum = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = lane * 4 + k;
        v[k] = r < R ? sm.rowcnt[r] : 0u;
        sum += v[k];
      }
      uint32_t x = sum;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      uint32_t run = x - sum;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = lane * 4 + k;
        if (r < R) rowoff[r0 + r] = run;
        run += v[k];
      }
    }
    if (threadIdx.x == 0) usub[g] = U;
    heavy_sync();
  }
}

// ---- the split of the first kHeavyPar listed sub-buckets, by many workgroups.  Their
// pairs are cut into chunks of kSplitChunk (a sub-bucket's last chunk shorter); each
// workgroup takes chunks j = blockIdx.x, blockIdx.x + gridDim.x, ...  in list order.
constexpr uint32_t kSplitChunk = 8192;

// the listed sub-buckets' pair ranges and chunk prefix in LDS (npar <= kHeavyPar)
__device__ __forceinline__ void heavy_chunk_table(const uint32_t* sbb, const uint32_t* ov_list, uint32_t npar,
                                                  uint32_t* s_beg, uint32_t* s_end, uint32_t* s_c0) {
  if (threadIdx.x < 64) {
    const uint32_t it = threadIdx.x;
    uint32_t a = 0, b = 0;
    if (it < npar) {
      const uint32_t g = ov_list[it];
      a = sbb[g];
      b = sbb[g + 1];
    }
    const uint32_t nc = (b - a + kSplitChunk - 1) / kSplitChunk;
    uint32_t x = nc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if ((int)it >= d) x += y;
    }
    s_beg[it] = a;
    s_end[it] = b;
    s_c0[it + 1] = x;
    if (it == 0) s_c0[0] = 0u;
  }
  __syncthreads();
}

// the sub-bucket of chunk j (j below the chunk total): the last it with s_c0[it] <= j
__device__ __forceinline__ uint32_t heavy_chunk_owner(const uint32_t* s_c0, uint32_t j) {
  uint32_t lo = 0, n = kHeavyPar;
#pragma unroll
  for (int s = 0; s < 6; ++s) {  // kHeavyPar = 2^6 candidates
    const uint32_t half = n >> 1;
    if (s_c0[lo + half] <= j) lo += half;
    n -= half;
  }
  return lo;
}

// Calls f(it, a, b) for each chunk [a, b) of this workgroup, it its sub-bucket's place
// in the list.  f is called by all threads and may use barriers.
template <typename Fn>
__device__ __forceinline__ void heavy_chunks(const uint32_t* sbb, const uint32_t* ov_list, uint32_t npar, Fn f) {
  __shared__ uint32_t s_beg[kHeavyPar], s_end[kHeavyPar], s_c0[kHeavyPar + 1];
  heavy_chunk_table(sbb, ov_list, npar, s_beg, s_end, s_c0);
  const uint32_t nch = s_c0[kHeavyPar];
  for (uint32_t j = blockIdx.x; j < nch; j += gridDim.x) {
    const uint32_t it = heavy_chunk_owner(s_c0, j);
    const uint32_t a = s_beg[it] + (j - s_c0[it]) * kSplitChunk;
    const uint32_t b = s_end[it] - a > kSplitChunk ? a + kSplitChunk : s_end[it];
    f(it, a, b);
  }
}

// A wave's keys of one LDS counter combined (heavy_hot) into count[x(k)].
template <typename X>
__device__ __forceinline__ void heavy_count(const uint32_t* key, uint32_t a, uint32_t b, uint32_t* count, X x) {
  const int lane = threadIdx.x & 63;
  heavy_stream<false, uint32_t>(key, nullptr, a, b, [&](uint32_t k, uint32_t, bool ok) {
    const uint32_t d = ok ? x(k) : 0u;
    uint32_t hot;
    const uint64_t m = heavy_hot(d, ok, hot);
    if (ok && !((m >> lane) & 1ull)) atomicAdd(&count[d], 1u);
    if (lane == 0 && m) atomicAdd(&count[hot], (uint32_t)__popcll(m));
  });
}

// pairs of each row of the listed sub-buckets
__global__ __launch_bounds__(kHeavyThreads) void k_heavy_rows(const uint32_t* __restrict__ ikey,
                                                              const uint32_t* __restrict__ sbb, int colbits,
                                                              const uint32_t* __restrict__ ov_list,
                                                              const uint32_t* __restrict__ ov_count,
                                                              uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_rows[kHvyRows];
  const uint32_t n_over = *ov_count;
  const uint32_t npar = n_over < (uint32_t)kHeavyPar ? n_over : (uint32_t)kHeavyPar;
  if (npar == 0) return;
  heavy_chunks(sbb, ov_list, npar, [&](uint32_t it, uint32_t a, uint32_t b) {
    for (int r = threadIdx.x; r < kHvyRows; r += kHeavyThreads) s_rows[r] = 0u;
    __syncthreads();
    heavy_count(ikey, a, b, s_rows, [&](uint32_t k) { return k >> colbits; });
    __syncthreads();
    const HeavyTable t(hvy, it);
    for (int r = threadIdx.x; r < kHvyRows; r += kHeavyThreads) {
      const uint32_t c = s_rows[r];
      if (c) atomicAdd(&t.rpair[r], c);
    }
    __syncthreads();
  });
}

// one workgroup (kHvyRows threads) per listed sub-bucket: the digits of each row, the
// digit counts cleared
__global__ __launch_bounds__(kHvyRows) void k_heavy_layout(const uint32_t* __restrict__ sbb, int colbits,
                                                           const uint32_t* __restrict__ ov_list,
                                                           const uint32_t* __restrict__ ov_count,
                                                           uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_scan[kHvyRows / 64 + 1];
  const uint32_t n_over = *ov_count;
  const uint32_t it = blockIdx.x;
  if (it >= n_over || it >= (uint32_t)kHeavyPar) return;
  const HeavyTable t(hvy, it);
  const uint32_t g = ov_list[it];
  const uint64_t n = sbb[g + 1] - sbb[g];
  const int r = threadIdx.x;
  const uint32_t c = t.rpair[r];
  const int lg_max = colbits > 12 ? colbits - 12 : 0;  // digits no narrower than a leaf
  const int lg_min = colbits > 23 ? colbits - 23 : 0;  // nor wider than 2^23 keys
  int lg = 0;
  if (c) {
    const uint64_t q = (uint64_t)c * kHvyShare / n;
    lg = q > 1 ? 63 - __clzll((long long)q) : 0;
    lg = lg < lg_min ? lg_min : (lg > lg_max ? lg_max : lg);
  }
  const uint32_t nr = c ? 1u << lg : 0u;
  uint32_t total;
  const uint32_t base = block_scan_u32(nr, s_scan, &total);
  t.rbase[r] = base;
  t.rsh[r] = (uint32_t)(colbits - lg);
  if (r == 0) {
    t.rbase[kHvyRows] = total;
    t.meta[0] = total;
  }
  for (uint32_t d = threadIdx.x; d < total; d += kHvyRows) t.hist[d] = 0u;
}

// a sub-bucket's digit layout into LDS (s_rbase: kHvyRows + 1 words, s_rsh: kHvyRows)
__device__ __forceinline__ void heavy_load_layout(const HeavyTable& t, uint32_t* s_rbase, uint32_t* s_rsh) {
  for (int r = threadIdx.x; r <= kHvyRows; r += blockDim.x) {
    s_rbase[r] = t.rbase[r];
    if (r < kHvyRows) s_rsh[r] = t.rsh[r];
  }
}

// pairs per first-level digit, summed over the chunks into the table's hist
__global__ __launch_bounds__(kHeavyThreads) void k_heavy_hist(const uint32_t* __restrict__ ikey,
                                                              const uint32_t* __restrict__ sbb, int colbits,
                                                              const uint32_t* __restrict__ ov_list,
                                                              const uint32_t* __restrict__ ov_count,
                                                              uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_hist[kHvyDigits];
  __shared__ uint32_t s_rbase[kHvyRows + 1], s_rsh[kHvyRows];
  const uint32_t n_over = *ov_count;
  const uint32_t npar = n_over < (uint32_t)kHeavyPar ? n_over : (uint32_t)kHeavyPar;
  if (npar == 0) return;
  heavy_chunks(sbb, ov_list, npar, [&](uint32_t it, uint32_t a, uint32_t b) {
    const HeavyTable t(hvy, it);
    heavy_load_layout(t, s_rbase, s_rsh);
    for (int d = threadIdx.x; d < kHvyDigits; d += kHeavyThreads) s_hist[d] = 0u;
    __syncthreads();
    const uint32_t nd = s_rbase[kHvyRows];
    heavy_count(ikey, a, b, s_hist, [&](uint32_t k) { return heavy_digit(k, colbits, s_rbase, s_rsh); });
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += kHeavyThreads) {
      const uint32_t c = s_hist[d];
      if (c) atomicAdd(&t.hist[d], c);
    }
    __syncthreads();
  });
}

// one workgroup per listed sub-bucket: the digit starts (absolute pair positions) from
// the digit counts, which become the scatter's cursors; digit ranges no wider than a
// leaf with more than kBigLeafPairs pairs are listed as big leaves
__global__ __launch_bounds__(kHeavyThreads) void k_heavy_starts(const uint32_t* __restrict__ sbb, int colbits,
                                                                const uint32_t* __restrict__ ov_list,
                                                                const uint32_t* __restrict__ ov_count,
                                                                uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_off[kHvyDigits];
  __shared__ uint32_t s_scan[kHeavyThreads / 64 + 1];
  const uint32_t n_over = *ov_count;
  const uint32_t it = blockIdx.x;
  if (it >= n_over || it >= (uint32_t)kHeavyPar) return;
  const HeavyTable t(hvy, it);
  const uint32_t nd = t.meta[0];
  const uint32_t g = ov_list[it];
  const uint32_t beg = sbb[g], end = sbb[g + 1];
  for (uint32_t d = threadIdx.x; d < nd; d += kHeavyThreads) s_off[d] = t.hist[d];
  __syncthreads();
  block_scan_array(s_off, (int)nd, s_scan);  // (ends with a barrier)
  const BigLeaves big(hvy);
  for (uint32_t d = threadIdx.x; d < nd; d += kHeavyThreads) {
    const uint32_t a = beg + s_off[d], b = d + 1 < nd ? beg + s_off[d + 1] : end;
    t.st[d] = a;
    t.hist[d] = a;
    if (b - a > kBigLeafPairs) {
      // the row of digit d: the last r with rbase[r] <= d (rare: read from the table)
      uint32_t r = 0, n = kHvyRows;
      for (int s = 0; s < 8; ++s) {
        const uint32_t half = n >> 1;
        if (t.rbase[r + half] <= d) r += half;
        n -= half;
      }
      const uint32_t sh = t.rsh[r];
      if ((1u << sh) <= (uint32_t)kLeafKeys) {
        const uint32_t i = atomicAdd(big.list, 1u);
        if (i < (uint32_t)kBigLeaves) {
          uint32_t* const q = big.rec(i);
          q[0] = it;
          q[1] = d;
          q[2] = a;
          q[3] = b;
          q[4] = (r << colbits) + ((d - t.rbase[r]) << sh);
        }
      }
    }
  }
  if (threadIdx.x == 0) t.st[nd] = end;
}

// each chunk's pairs moved from (ikey, ival) to (akey, aval) in first-level digit order:
// the chunk's digit counts taken again, a block of each digit reserved from the table's
// cursors, then each pair placed in its digit's block
template <typename V>
__global__ __launch_bounds__(kHeavyThreads) void k_heavy_scatter(const uint32_t* __restrict__ ikey,
                                                                 const V* __restrict__ ival,
                                                                 uint32_t* __restrict__ akey, V* __restrict__ aval,
                                                                 const uint32_t* __restrict__ sbb, int colbits,
                                                                 const uint32_t* __restrict__ ov_list,
                                                                 const uint32_t* __restrict__ ov_count,
                                                                 uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_hist[kHvyDigits];
  __shared__ uint32_t s_rbase[kHvyRows + 1], s_rsh[kHvyRows];
  const uint32_t n_over = *ov_count;
  const uint32_t npar = n_over < (uint32_t)kHeavyPar ? n_over : (uint32_t)kHeavyPar;
  if (npar == 0) return;
  const int lane = threadIdx.x & 63;
  {  // the big leaves' accumulators cleared (k_heavy_bigleaf adds into them next)
    const BigLeaves big(hvy);
    uint32_t* const acc = big.list + kBigListWords;
    const size_t nw = (size_t)big.count() * kBigAccWords;
    for (size_t w = (size_t)blockIdx.x * kHeavyThreads + threadIdx.x; w < nw; w += (size_t)gridDim.x * kHeavyThreads)
      acc[w] = 0u;
  }
  heavy_chunks(sbb, ov_list, npar, [&](uint32_t it, uint32_t a, uint32_t b) {
    const HeavyTable t(hvy, it);
    heavy_load_layout(t, s_rbase, s_rsh);
    for (int d = threadIdx.x; d < kHvyDigits; d += kHeavyThreads) s_hist[d] = 0u;
    __syncthreads();
    const uint32_t nd = s_rbase[kHvyRows];
    heavy_count(ikey, a, b, s_hist, [&](uint32_t k) { return heavy_digit(k, colbits, s_rbase, s_rsh); });
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += kHeavyThreads) {
      const uint32_t c = s_hist[d];
      s_hist[d] = c ? atomicAdd(&t.hist[d], c) : 0u;
    }
    __syncthreads();
    heavy_stream<true, V>(ikey, ival, a, b, [&](uint32_t k, V v, bool ok) {
      const uint32_t d = ok ? heavy_digit(k, colbits, s_rbase, s_rsh) : 0u;
      uint32_t hot;
      const uint64_t m = heavy_hot(d, ok, hot);
      uint32_t base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_hist[hot], (uint32_t)__popcll(m));
      base = __shfl(base, 0, 64);
      const bool mine = (m >> lane) & 1ull;
      uint32_t pos = 0;
      if (mine)
        pos = base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
      else if (ok)
        pos = atomicAdd(&s_hist[d], 1u);
      if (ok) {
        akey[pos] = k;
        aval[pos] = v;
      }
    });
    __syncthreads();
  });
}

// the rounds of the listed big leaves, one per workgroup at a time, added into their
// accumulators (each leaf's pairs in (akey, aval) [a, b), keys from k0)
template <typename V>
__global__ __launch_bounds__(kHeavyThreads) void k_heavy_bigleaf(const uint32_t* akey, const V* aval,
                                                                 const uint32_t* __restrict__ emax,
                                                                 const uint32_t* __restrict__ ov_count,
                                                                 uint32_t* __restrict__ hvy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const HeavySmem sm(smem);
  __shared__ uint32_t s_p0[kBigLeaves + 1];
  if (*ov_count == 0) return;
  const BigLeaves big(hvy);
  const uint32_t nbig = big.count();
  if (nbig == 0) return;
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (uint32_t i = 0; i < nbig; ++i) {
      s_p0[i] = s;
      s += (big.rec(i)[3] - big.rec(i)[2] + kRound - 1) / kRound;
    }
    s_p0[nbig] = s;
  }
  for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
    sm.lo[h] = 0ull;
    sm.hi[h] = 0ll;
    sm.top[h] = 0ll;
  }
  if (threadIdx.x < kLeafKeys / 4) ((uint32_t*)sm.occ)[threadIdx.x] = 0u;
  __syncthreads();
  const int F = 1117 - (int)*emax;
  for (uint32_t p = blockIdx.x; p < s_p0[nbig]; p += gridDim.x) {
    uint32_t i = 0;
    while (i + 1 < nbig && s_p0[i + 1] <= p) ++i;
    const uint32_t* const q = big.rec(i);
    const uint32_t a = q[2] + (p - s_p0[i]) * kRound;
    const uint32_t b = q[3] - a > kRound ? a + kRound : q[3];
    heavy_leaf_sum<V>(sm, akey, aval, a, b, q[4], F);
    unsigned long long* const glo = big.lo(i);
    unsigned long long* const ghi = big.hi(i);
    unsigned long long* const gtop = big.top(i);
    uint32_t* const gocc = big.occ(i);
    for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
      if (!sm.occ[h]) continue;
      atomicAdd(&glo[h], sm.lo[h]);
      atomicAdd(&ghi[h], (unsigned long long)sm.hi[h]);
      atomicAdd(&gtop[h], (unsigned long long)sm.top[h]);
      gocc[h] = 1u;
      sm.lo[h] = 0ull;
      sm.hi[h] = 0ll;
      sm.top[h] = 0ll;
    }
    __syncthreads();
    if (threadIdx.x < kLeafKeys / 4) ((uint32_t*)sm.occ)[threadIdx.x] = 0u;
    __syncthreads();
  }
}

// The first-level digit ranges of the first kHeavyPar listed sub-buckets, split by
// k_heavy_scatter: range d0 of sub-bucket it is reduced by workgroup d0 mod gridDim.x,
// its entries written from its own first pair's place (its pairs all read before;
// other workgroups read other ranges), its entry count recorded in the table and added
// to its row's.
template <typename V, bool RES = false>
__global__ __launch_bounds__(kHeavyThreads) void k_pass3_heavy_ranges(uint32_t* ikey, V* ival, uint32_t* akey,
                                                                    V* aval, int colbits,
                                                                    const uint32_t* __restrict__ emax,
                                                                    V* __restrict__ tres,
                                                                    const uint32_t* __restrict__ ov_count,
                                                                    uint32_t* __restrict__ hvy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const HeavySmem sm(smem);
  const uint32_t n_over = *ov_count;
  const uint32_t npar = n_over < (uint32_t)kHeavyPar ? n_over : (uint32_t)kHeavyPar;
  if (npar == 0) return;
  for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
    sm.lo[h] = 0ull;
    sm.hi[h] = 0ll;
    sm.top[h] = 0ll;
  }
  if (threadIdx.x < kLeafKeys / 4) ((uint32_t*)sm.occ)[threadIdx.x] = 0u;
  for (int r = threadIdx.x; r < 256; r += kHeavyThreads) sm.rowcnt[r] = 0u;
  __syncthreads();
  const int F = 1117 - (int)*emax;
  int32_t* const tcol = (int32_t*)akey;
  // the layout of the sub-bucket in hand, in the first of the two split-start arrays
  // (heavy_range uses the second)
  uint32_t* const s_rbase = sm.start;
  uint32_t* const s_rsh = sm.start + kHvyRows + 1;
  static_assert(2 * kHvyRows + 1 <= kDigits + 1, "the row layout fits one split-start array");
  // the big leaves (summed by k_heavy_bigleaf): their sub-bucket and digit
  __shared__ uint32_t s_big[2 * kBigLeaves];
  const BigLeaves big(hvy);
  const uint32_t nbig = big.count();
  if (threadIdx.x < nbig) {
    s_big[2 * threadIdx.x] = big.rec(threadIdx.x)[0];
    s_big[2 * threadIdx.x + 1] = big.rec(threadIdx.x)[1];
  }
  for (uint32_t it = 0; it < npar; ++it) {
    const HeavyTable t(hvy, it);
    heavy_load_layout(t, s_rbase, s_rsh);
    __syncthreads();
    const uint32_t nd0 = s_rbase[kHvyRows];
    for (uint32_t d0 = blockIdx.x; d0 < nd0; d0 += gridDim.x) {
      const uint32_t a = t.st[d0], b = t.st[d0 + 1];
      if (a == b) {  // (its count word still holds the scatter's cursor)
        if (threadIdx.x == 0) t.ucnt[d0] = 0u;
        continue;
      }
      uint32_t r = 0, n = kHvyRows;  // the row of digit d0: the last r with s_rbase[r] <= d0
#pragma unroll
      for (int s = 0; s < 8; ++s) {  // kHvyRows = 2^8 candidates
        const uint32_t half = n >> 1;
        if (s_rbase[r + half] <= d0) r += half;
        n -= half;
      }
      const uint32_t sh = s_rsh[r];
      const uint32_t k0 = (r << colbits) + ((d0 - s_rbase[r]) << sh);
      uint32_t bi = nbig;
      for (uint32_t i = 0; i < nbig; ++i)
        if (s_big[2 * i] == it && s_big[2 * i + 1] == d0) bi = i;
      uint32_t U;
      if (bi < nbig) {  // summed already: its accumulated sums carried once more
        const unsigned long long* const glo = big.lo(bi);
        const unsigned long long* const ghi = big.hi(bi);
        const unsigned long long* const gtop = big.top(bi);
        const uint32_t* const gocc = big.occ(bi);
        for (int h = threadIdx.x; h < kLeafKeys; h += kHeavyThreads) {
          if (!gocc[h]) continue;
          sm.lo[h] = glo[h];
          sm.hi[h] = (long long)ghi[h];
          sm.top[h] = (long long)gtop[h];
          sm.occ[h] = 1;
        }
        __syncthreads();
        heavy_normalise(sm);
        __syncthreads();
        U = heavy_leaf_emit<V, RES>(sm, k0, F, colbits, tcol + a, aval + a, RES ? tres + a : nullptr, 0);
      } else {
        U = heavy_range<V, RES>(sm, ikey, ival, akey, aval, a, b, k0, 1u << sh, F, colbits, tcol + a, aval + a,
                                RES ? tres + a : nullptr, 0);
      }
      if (threadIdx.x == 0) {
        t.ucnt[d0] = U;
        atomicAdd(&t.rcnt[r], U);
      }
    }
    __syncthreads();  // (the next layout overwrites this one)
  }
}

// last index d in [0, n) with off[d] <= f (off nondecreasing, off[0] <= f)
template <typename P>
__device__ __forceinline__ uint32_t heavy_find(P off, uint32_t n, uint32_t f) {
  uint32_t lo = 0;
  while (n > 1) {
    const uint32_t half = n >> 1;
    if (off[lo + half] <= f) lo += half;
    n -= half;
  }
  return lo;
}

constexpr uint32_t kFinalWave = 4096;  // entries one wavefront of k_final copies

// One workgroup per sub-bucket of the table: its ranges' entry counts replaced by their
// offsets (k_final_heavy gathers the entries from the ranges through them), the row
// offsets within the sub-bucket and its entry count.  A sub-bucket of at most
// kFinalWave entries, which k_final copies as one run from its first pair's place, has
// them moved there: each thread reads its entries, and writes them after a barrier.
constexpr int kFinishThreads = 1024;
template <typename V, bool RES = false>
__global__ __launch_bounds__(kFinishThreads) void k_pass3_heavy_finish(uint32_t* akey, V* aval, V* tres,
                                                                     const uint32_t* __restrict__ sbb, int s2,
                                                                     int64_t n_node, uint32_t* __restrict__ rowoff,
                                                                     uint32_t* __restrict__ usub,
                                                                     const uint32_t* __restrict__ ov_list,
                                                                     const uint32_t* __restrict__ ov_count,
                                                                     uint32_t* __restrict__ hvy) {
  __shared__ uint32_t s_off[kHvyDigits];
  __shared__ uint32_t s_scan[kFinishThreads / 64 + 1];
  const uint32_t n_over = *ov_count;
  const uint32_t it = blockIdx.x;
  if (it >= n_over || it >= (uint32_t)kHeavyPar) return;
  const HeavyTable t(hvy, it);
  const uint32_t nd0 = t.meta[0];
  const int64_t g = ov_list[it];
  const uint32_t beg = sbb[g];
  for (uint32_t d = threadIdx.x; d < nd0; d += kFinishThreads) s_off[d] = t.ucnt[d];
  __syncthreads();
  const uint32_t U = block_scan_array(s_off, (int)nd0, s_scan);  // (ends with a barrier)
  for (uint32_t d = threadIdx.x; d < nd0; d += kFinishThreads) t.ucnt[d] = s_off[d];
  int32_t* const tcol = (int32_t*)akey;
  if (U <= kFinalWave) {
    constexpr int PER = kFinalWave / kFinishThreads;
    int32_t c[PER];
    V v[PER], e[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t f = j * kFinishThreads + threadIdx.x;
      if (f >= U) continue;
      const uint32_t d = heavy_find(s_off, nd0, f);
      const uint32_t src = t.st[d] + (f - s_off[d]);
      c[j] = tcol[src];
      v[j] = aval[src];
      if constexpr (RES) e[j] = tres[src];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t f = j * kFinishThreads + threadIdx.x;
      if (f >= U) continue;
      tcol[beg + f] = c[j];
      aval[beg + f] = v[j];
      if constexpr (RES) tres[beg + f] = e[j];
    }
  }
  // row offsets within the sub-bucket from the entries per row
  const int64_t r0 = g << s2;
  const int R = (int)min((int64_t)1 << s2, n_node - r0);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = lane * 4 + k;
      v[k] = r < R ? t.rcnt[r] : 0u;
      sum += v[k];
    }
    uint32_t x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    uint32_t run = x - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = lane * 4 + k;
      if (r < R) rowoff[r0 + r] = run;
      run += v[k];
    }
  }
  if (threadIdx.x == 0) usub[g] = U;
}

// ------------------------------------------------------------------------- final
// One wavefront per sub-bucket g: its entries copied to their final place ubase[g],
// its rows' row_ptr = ubase[g] + local row offset.
// GROUPED (running sums of a grouped build): also each entry's residual (tres -> res)
// and its row (rows), the form in which the next group's pass reads them back.
template <typename V, bool GROUPED = false>
__global__ __launch_bounds__(256) void k_final(const uint32_t* __restrict__ sbb, const uint32_t* __restrict__ ubase,
                                               const int32_t* __restrict__ tcol, const V* __restrict__ tval,
                                               const V* __restrict__ tres, const uint32_t* __restrict__ rowoff,
                                               int s2, int64_t n_node, int64_t nsub, int32_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ col_idx, V* __restrict__ vals,
                                               V* __restrict__ res, int32_t* __restrict__ rows, int64_t cap,
                                               uint32_t* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (g >= nsub) return;
  const int64_t nnz = ubase[nsub];
  const uint32_t base = ubase[g], U = ubase[g + 1] - base;
  const int64_t r0 = g << s2;
  const int R = (int)min((int64_t)1 << s2, n_node - r0);
  if (nnz <= cap && U <= kFinalWave) {  // (larger: a heavy sub-bucket, k_final_heavy)
    const uint32_t src = sbb[g];
    for (uint32_t f = lane; f < U; f += 64) {
      col_idx[base + f] = tcol[src + f];
      vals[base + f] = tval[src + f];
      if constexpr (GROUPED) res[base + f] = tres[src + f];
    }
    if constexpr (GROUPED) {
      for (int r = lane; r < R; r += 64) {
        const uint32_t k1 = r + 1 < R ? rowoff[r0 + r + 1] : U;
        for (uint32_t k = rowoff[r0 + r]; k < k1; ++k) rows[base + k] = (int32_t)(r0 + r);
      }
    }
  } else if (nnz > cap && g == 0 && lane == 0) {
    raise_flag(status, KB_F_CAPACITY);
  }
  for (int r = lane; r < R; r += 64) row_ptr[r0 + r] = (int32_t)(base + rowoff[r0 + r]);
  if (g == nsub - 1 && lane == 0) row_ptr[n_node] = (int32_t)nnz;
}

// The entries of the sub-buckets k_final leaves (more than kFinalWave: only a heavy
// sub-bucket, listed by pass 3, can hold more than a pass-3 table), copied by all the
// workgroups of the grid in chunks of 1024: from the sub-bucket's first pair's place
// on, or, for the first kHeavyPar listed, from the digit ranges that hold them (entry f
// of the range d whose entry offset is the last at or below f, at the range's start
// plus f minus that offset).  With GROUPED each entry's row is found by a binary search
// of the sub-bucket's row offsets.
template <typename V, bool GROUPED = false>
__global__ __launch_bounds__(256) void k_final_heavy(const uint32_t* __restrict__ sbb, const uint32_t* __restrict__ ubase,
                                                     const int32_t* __restrict__ tcol, const V* __restrict__ tval,
                                                     const V* __restrict__ tres, const uint32_t* __restrict__ rowoff,
                                                     int s2, int64_t n_node, int64_t nsub,
                                                     const uint32_t* __restrict__ ov_list,
                                                     const uint32_t* __restrict__ ov_count,
                                                     const uint32_t* __restrict__ hvy,
                                                     int32_t* __restrict__ col_idx, V* __restrict__ vals,
                                                     V* __restrict__ res, int32_t* __restrict__ rows, int64_t cap) {
  __shared__ uint32_t s_off[kHvyDigits];  // entry offsets of the ranges
  const uint32_t n_over = *ov_count;
  if (n_over == 0 || (int64_t)ubase[nsub] > cap) return;
  for (uint32_t it = 0; it < n_over; ++it) {
    const int64_t g = ov_list[it];
    const uint32_t base = ubase[g], U = ubase[g + 1] - base;
    if (U <= kFinalWave) continue;
    const uint32_t beg = sbb[g];
    const bool ranged = it < (uint32_t)kHeavyPar;
    const HeavyTable t(const_cast<uint32_t*>(hvy), ranged ? it : 0u);
    const uint32_t nd0 = ranged ? t.meta[0] : 0u;
    if (ranged) {
      __syncthreads();  // (the previous sub-bucket's offsets are no longer read)
      for (uint32_t d = threadIdx.x; d < nd0; d += blockDim.x) s_off[d] = t.ucnt[d];
      __syncthreads();
    }
    const int64_t r0 = g << s2;
    const int R = (int)min((int64_t)1 << s2, n_node - r0);
    for (uint32_t c = blockIdx.x * 1024u; c < U; c += gridDim.x * 1024u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t f = c + j * 256 + threadIdx.x;
        if (f >= U) continue;
        uint32_t src = beg + f;
        if (ranged) {
          const uint32_t d = heavy_find(s_off, nd0, f);
          src = t.st[d] + (f - s_off[d]);
        }
        col_idx[base + f] = tcol[src];
        vals[base + f] = tval[src];
        if constexpr (GROUPED) {
          res[base + f] = tres[src];
          int lo = 0, hi = R - 1;  // last row whose first entry is at or before f
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rowoff[r0 + mid] <= f)
              lo = mid;
            else
              hi = mid - 1;
          }
          rows[base + f] = (int32_t)(r0 + lo);
        }
      }
    }
  }
}

}  // namespace kb
