// kb_api.hip -- host side of the C ABI declared in include/kbuild.h.
//
// Validates arguments, carves the caller's workspace and enqueues the kernel
// sequence on the caller's stream.  Allocates nothing and keeps no state.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>

#include "kb_adjoint.hpp"
#include "kb_assemble.hpp"
#include "kb_batch.hpp"
#include "kb_kernels.hpp"
#include "kbuild.h"

namespace {

using namespace kb;

constexpr size_t kAlign = 256;
constexpr float kDefaultTau = 16.0f;
constexpr int kDefaultBlock = 256;
// pairs per pass-2 segment: the short one keeps three scatter workgroups per CU, the long
// one (one per CU) is taken for tetrahedra when a segment would otherwise give runs of
// fewer than kMinRun pairs per sub-bucket (measured: 18% faster scatter on the 20M-tet
// mesh, 35% slower on brick meshes with the same sub-bucket counts)
constexpr int kSeg = 4096, kSegLong = 8192, kMinRun = 16;
constexpr int kSegThreads = 512;   // threads per pass-2 scatter workgroup
constexpr int kTargetBuckets = 256;  // first-level buckets (pass-1 run length)
constexpr double kSubEntries = 300;   // target distinct entries per sub-bucket
constexpr int kHTMin = 512, kHTMax = 4096;
constexpr int kHeavyGrid = 64;  // workgroups of k_pass3_heavy (each takes whole sub-buckets)
static_assert(kHeavyGrid >= kHeavyPar, "k_pass3_heavy's first kHeavyPar workgroups clear the split tables");
constexpr unsigned kFinalHeavyGrid = 256;  // workgroups copying the entries of heavy sub-buckets
constexpr double kHalfTileRatio = 16;   // pairs per tile x bucket histogram entry
constexpr size_t kWideStage = 112640;  // staged pair bytes per pass-1 tile, elements of > 8 rows

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Plan {
  int nen = 0, te = 0, prec = 0, block = kDefaultBlock;
  int op = KB_OP_STIFFNESS;            // element integrand
  int dof = 1;                         // degrees of freedom per node (assembly only)
  float tau = kDefaultTau;
  int64_t nel = 0, nn = 0, T = 0;
  size_t vbytes = 8;
  // assembly geometry
  int s1 = 0, s2 = 0, p2 = 1, nb = 0;  // bucket / sub-bucket shifts, sub-buckets per bucket, buckets
  int colbits = 1;                     // bits of a column index
  int ht = 2048;                       // pass-3 hash slots
  int seg = kSeg;                      // pairs per pass-2 segment
  int tile = 0;                        // elements (= threads) per pass-1 workgroup
  int cus = 256;                       // compute units of the current device (launch time)
  int64_t ntiles = 0, nsub = 0, nhist = 0, nseg_max = 0;
  int64_t csr_cap = 0, ntiles_csr = 0;  // running sums read back as pairs (grouped builds)
  size_t lds1 = 0, lds2 = 0;
  // workspace offsets
  size_t o_coords4 = 0, o_hist = 0, o_csum = 0, o_tot = 0, o_part = 0, o_total = 0, o_bstart = 0, o_segbase = 0, o_hist2 = 0, o_seg2b = 0, o_emax = 0,
         o_dconn = 0, o_ovl = 0, o_hvy = 0, o_tres = 0, o_row1 = 0, o_col1 = 0, o_val1 = 0, o_key2 = 0, o_val2 = 0, o_sbb = 0, o_rowoff = 0, o_usub = 0, o_ubase = 0,
         total = 0;
};

// compute units of the current device, cached per device ordinal
int device_cus(int* out) {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KB_EHIP;
  if (dev >= 0 && dev < 64) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) {
      *out = c;
      return KB_OK;
    }
  }
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return KB_EHIP;
  if (dev >= 0 && dev < 64) cache[dev].store(n, std::memory_order_relaxed);
  *out = n;
  return KB_OK;
}

int ilog2_ceil(int64_t x) {
  int k = 0;
  while (((int64_t)1 << k) < x) ++k;
  return k;
}

// dof > 1: element matrices with dof components per node are assembled as elements of
// nen * dof "nodes" (global DOF dof * E_a + i); nen and nn below are those of that view
// csr_cap > 0: each pass also reads back up to csr_cap entries of running sums as two
// pairs each (value and residual), and writes residuals (grouped builds)
int make_plan(const kb_mesh* m, int prec, const kb_tuning* tu, Plan* p, int dof = 1, int64_t csr_cap = 0) {
  if (!m) return KB_EINVAL;
  if (m->elem != KB_HEX8 && m->elem != KB_TET4) return KB_EINVAL;
  if (prec != KB_FP64 && prec != KB_FP32 && prec != KB_FP32_FB64) return KB_EINVAL;
  if (m->n_elem < 0 || m->n_node < 0 || (m->op != KB_OP_STIFFNESS && m->op != KB_OP_MASS)) return KB_EINVAL;
  if (dof < 1 || dof > 3) return KB_EINVAL;
  p->op = m->op;
  p->dof = dof;
  p->nen = m->elem * dof;
  p->te = p->nen * (p->nen + 1) / 2;
  p->prec = prec;
  p->nel = m->n_elem;
  if (m->n_node >= (int64_t)INT32_MAX / dof) return KB_ERANGE;
  p->nn = m->n_node * dof;
  if (p->nn >= (int64_t)INT32_MAX) return KB_ERANGE;
  if (csr_cap < 0) return KB_EINVAL;
  if (p->nel > (int64_t)INT32_MAX / p->te || csr_cap > ((int64_t)INT32_MAX - p->nel * p->te) / 2) return KB_ERANGE;
  p->csr_cap = csr_cap;
  p->T = p->nel * p->te + 2 * csr_cap;  // pairs of one pass
  p->vbytes = prec == KB_FP64 ? 8 : 4;
  int bucket_bits = 0, sub_bits = 0;
  if (tu) {
    if (tu->block) {
      if (tu->block < 64 || tu->block > 1024 || (tu->block & 63)) return KB_EINVAL;
      p->block = tu->block;
    }
    if (tu->fb_tau != 0.0f) {
      if (!(tu->fb_tau > 1.0f)) return KB_EINVAL;
      p->tau = tu->fb_tau;
    }
    if (tu->sub_bits < 0 || tu->sub_bits > 8 || tu->bucket_bits < 0 || tu->bucket_bits > 16) return KB_EINVAL;
    if (tu->bucket_bits && tu->sub_bits && tu->sub_bits > tu->bucket_bits) return KB_EINVAL;
    bucket_bits = tu->bucket_bits;
    sub_bits = tu->sub_bits;
    if (tu->seg_pairs != 0 && tu->seg_pairs != kSeg && tu->seg_pairs != kSegLong) return KB_EINVAL;
    if (tu->table_slots != 0 && (tu->table_slots < kHTMin || tu->table_slots > kHTMax ||
                                 (tu->table_slots & (tu->table_slots - 1))))
      return KB_EINVAL;
  }
  // sub-buckets: about a third of the pass-3 hash table of distinct entries on average;
  // distinct entries per row estimated from the pairs per row and the typical number
  // of elements sharing an entry (about 7 for tetrahedra, 2.5 for bricks)
  p->colbits = 1;
  while (((int64_t)1 << p->colbits) < p->nn) ++p->colbits;
  // (running sums read back bring up to csr_cap distinct entries of their own)
  const double avg = p->nn > 0 ? (double)(p->nel * p->te) / (double)p->nn : 1.0;
  const double u_row = std::max(1.0, avg / (m->elem == KB_TET4 ? 7.4 : 2.5) +
                                         (p->nn > 0 ? (double)csr_cap / (double)p->nn : 0.0));
  const int s2_max = std::min(8, 31 - p->colbits);
  if (sub_bits) {
    if (sub_bits > s2_max) return KB_EINVAL;
    p->s2 = sub_bits;
  } else {
    int s2 = 0;
    while (s2 < s2_max && ((double)(1 << (s2 + 1))) * u_row <= kSubEntries) ++s2;
    p->s2 = s2;
  }
  // hash slots: about four per expected distinct entry (short probe chains)
  p->ht = kHTMin;
  while (p->ht < kHTMax && p->ht < 4.0 * (double)(1 << p->s2) * u_row) p->ht *= 2;
  if (bucket_bits) {
    p->s1 = bucket_bits < p->s2 ? p->s2 : bucket_bits;
  } else {
    const int64_t nsub_min = div_up(p->nn > 0 ? p->nn : 1, (int64_t)1 << p->s2);
    int d = ilog2_ceil(div_up(nsub_min, kTargetBuckets));
    if (d > 10) d = 10;
    // rows are stored within their bucket in 16 bits: at most 2^16 rows per bucket
    p->s1 = std::min(16, p->s2 + d);
  }
  if (p->s1 - p->s2 > 10) return KB_EINVAL;
  // pass-1 staging per tile (bytes): the smallest tile the plan may take, and the scan words
  const size_t wide_tile = std::min<size_t>(256, std::max<size_t>(1, kWideStage / ((size_t)p->te * (8 + p->vbytes))));
  const size_t stage_min = p->nen <= 8 ? (size_t)(p->nen == 4 ? (prec == KB_FP64 ? 384 : 512) : 128) * p->te *
                                                 (8 + p->vbytes) + 4 * (2 * 512 / 64 + 2)
                                       : wide_tile * p->te * (8 + p->vbytes) + 4 * (kWideThreads / 64 + 2) +
                                             wide_tile * ((size_t)p->nen * 12 + 4) + 2 * (size_t)p->te;
  if (!bucket_bits && !sub_bits) {
    // very many rows: pass 1 keeps two LDS counters per bucket beside its staged pairs;
    // widen the buckets (beyond 1024 sub-buckets per bucket, the sub-buckets too) until
    // they fit beside the smallest tile
    // (the sub-bucket key packs the row within its sub-bucket beside the column in 31
    // bits, so the sub-buckets widen only up to s2_max: about 1.3e8 rows at most)
    while (p->s1 < 16 && stage_min + 8 * (size_t)div_up(p->nn, (int64_t)1 << p->s1) > 163840) {
      if (p->s1 + 1 - p->s2 > 10) {
        if (p->s2 + 1 > s2_max) break;
        ++p->s2;
        while (p->ht < kHTMax && p->ht < 4.0 * (double)(1 << p->s2) * u_row) p->ht *= 2;
      }
      ++p->s1;
    }
  }
  if (tu && tu->table_slots) p->ht = tu->table_slots;
  p->p2 = 1 << (p->s1 - p->s2);
  p->nb = (int)div_up(p->nn, (int64_t)1 << p->s1);
  p->nsub = (int64_t)p->nb * p->p2;
  // pass-1 tiles: pairs staged in LDS as (8-byte key, value).  Up to 8 rows: one
  // element per lane, `block` may pick the half-size tile (two workgroups per CU);
  // more rows (several DOFs per node): as many elements as keep the staged pairs near
  // 110 KB, on kWideThreads threads
  if (p->nen <= 8) {
    const int big = p->nen == 4 ? (prec == KB_FP64 ? 768 : 1024) : 256;
    const int small = big / 2 % 64 == 0 ? big / 2 : 64 * ((big / 2 + 63) / 64);
    // FP64 with 8 rows: the 256 tile's staged pairs take 147 KB; with more than about
    // 2000 buckets their counters no longer fit beside it, and a 192 tile takes over
    // (measured on the 27M bricks, FP64: 256 lanes, one wave on each SIMD, pass 1
    // 12.2 -> 9.5 ms against 192)
    const int mid = (p->nen == 8 && prec == KB_FP64) ? 192 : 0;
    auto lds_of = [&](int tile) {  // (scan words for up to two lanes per element)
      return (size_t)tile * p->te * (8 + p->vbytes) + 2 * 4 * (size_t)p->nb + 4 * (2 * (size_t)tile / 64 + 2);
    };
    p->tile = big;
    // bricks: the half tile (two workgroups per CU, one's gathers under the other's
    // writes) when the tile x bucket histogram it doubles stays small next to the pairs
    // (measured: randomly numbered 1M bricks 10% faster pass 1; the 256-brick batch, whose
    // histogram is 1/6 of its pairs, 4% slower overall)
    if (m->elem == KB_HEX8 && p->dof == 1 && p->nb > 0 &&
        (double)p->T >= kHalfTileRatio * (double)p->nb * (double)div_up(p->nel, small))
      p->tile = small;
    if (tu && (tu->block == big || tu->block == small || (mid && tu->block == mid))) p->tile = tu->block;
    if (mid && p->tile == big && lds_of(big) > 163840) p->tile = mid;
    if (lds_of(p->tile) > 163840) p->tile = small;  // many buckets: the counters need the room
    p->lds1 = lds_of(p->tile);
  } else {
    p->tile = (int)wide_tile;
    p->lds1 = (size_t)p->tile * p->te * (8 + p->vbytes) + 2 * 4 * (size_t)p->nb + 4 * (kWideThreads / 64 + 2) +
              (size_t)p->tile * p->nen * 12 + 4 * (size_t)p->tile + 2 * (size_t)p->te;
  }
  p->ntiles = div_up(p->nel, p->tile);
  p->ntiles_csr = div_up(csr_cap, kCsrTile);
  p->nhist = (int64_t)p->nb * (p->ntiles + p->ntiles_csr);
  if (csr_cap > 0 && 2 * (size_t)kCsrTile * (8 + p->vbytes) + 2 * 4 * (size_t)p->nb + 4 * (256 / 64 + 2) > 163840)
    return KB_EINVAL;
  if (tu && tu->seg_pairs)
    p->seg = tu->seg_pairs;
  else
    p->seg = (m->elem == KB_TET4 && (int64_t)kSeg < (int64_t)kMinRun * p->p2) ? kSegLong : kSeg;
  p->nseg_max = div_up(p->T, p->seg) + p->nb;
  p->lds2 = (size_t)p->seg * (p->vbytes + 4 + 2) + 2 * 4 * (size_t)p->p2 + 4 * (kSegThreads / 64 + 1);
  if (p->lds1 > 163840 || p->lds2 > 163840) return KB_EINVAL;
  size_t off = 0;
  auto take = [&](size_t bytes) {  // every region at least one aligned block
    size_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 1));
    return o;
  };
  const size_t T = (size_t)p->T;
  const int64_t scan_n = std::max<int64_t>(p->nb, p->nsub + 1);
  p->o_coords4 = take(p->dof > 1 ? 0 : 32 * (size_t)p->nn);  // assembly with several DOFs: no geometry
  // scan outputs hold n + 1 words: the scan writes its total after the last entry
  p->o_hist = take(4 * (size_t)p->nhist);
  p->o_csum = take(4 * (size_t)div_up(p->ntiles + p->ntiles_csr, kColChunk) * (size_t)p->nb);
  p->o_tot = take(4 * (size_t)p->nb);
  p->o_part = take(4 * (size_t)(div_up(scan_n, kScanChunk) + 1));
  p->o_total = take(8);
  p->o_bstart = take(4 * ((size_t)p->nb + 1));
  p->o_segbase = take(4 * ((size_t)p->nb + 1));
  p->o_hist2 = take(4 * (size_t)(p->nseg_max * p->p2));
  p->o_seg2b = take(4 * (size_t)p->nseg_max);
  p->o_emax = take(8);  // largest value exponent, then the count of heavy sub-buckets
  p->o_ovl = take(4 * (size_t)p->nsub);  // heavy sub-buckets (k_pass3_heavy)
  p->o_hvy = take(4 * ((size_t)kHeavyPar * kHvyWords + kBigWords));  // their split tables and big leaves
  p->o_dconn = take(p->dof > 1 ? 4 * (size_t)p->nen * (size_t)p->nel : 0);  // expanded connectivity
  p->o_tres = take(csr_cap > 0 ? p->vbytes * T : 0);  // residuals of the reduced entries
  p->o_row1 = take(2 * T);
  p->o_col1 = take(4 * T);
  p->o_val1 = take(p->vbytes * T);
  p->o_key2 = take(4 * T);
  p->o_val2 = take(p->vbytes * T);
  p->o_sbb = take(4 * ((size_t)p->nsub + 1));
  p->o_rowoff = take(4 * (size_t)p->nn);
  p->o_usub = take(4 * ((size_t)p->nsub + 1));
  p->o_ubase = take(4 * ((size_t)p->nsub + 1));
  p->total = off;
  return KB_OK;
}

struct Events {
  void** ev;
  hipStream_t s;
  int rec(int i) {
    if (!ev) return KB_OK;
    return hipEventRecord((hipEvent_t)ev[i], s) == hipSuccess ? KB_OK : KB_EHIP;
  }
};

#define KB_LAUNCH_CHECK()                                   \
  do {                                                      \
    if (hipGetLastError() != hipSuccess) return KB_EHIP;    \
  } while (0)
#define KB_TRY(x)                  \
  do {                             \
    int _r = (x);                  \
    if (_r != KB_OK) return _r;    \
  } while (0)

unsigned grid_for(int64_t n, int block) { return (unsigned)div_up(n, block); }

// exclusive scan in[0..n) -> out[0..n] (out holds n + 1 words), total64 optional
// (in-place allowed)
int scan(const int32_t* in, int64_t n, int32_t* part, int32_t* out, int64_t* total64, hipStream_t s) {
  if (n == 0) {
    k_scan_empty<<<1, 1, 0, s>>>(out, total64);
    KB_LAUNCH_CHECK();
    return KB_OK;
  }
  const int64_t nb = div_up(n, kScanChunk);
  k_scan_partials<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, part);
  KB_LAUNCH_CHECK();
  k_scan_top<<<1, kScanThreads, 0, s>>>(part, nb);
  KB_LAUNCH_CHECK();
  k_scan_down<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, part, out, total64);
  KB_LAUNCH_CHECK();
  return KB_OK;
}

template <typename K>
bool set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
         hipSuccess;
}

template <int NEN, Prec P, bool FROM_VALUES, int BLOCK, Op OP>
int launch_pass1_block(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, uint32_t* status,
                       hipStream_t s) {
  using V = typename PrecTraits<P>::V;
  if constexpr (NEN == 8 && !FROM_VALUES && OP == Op::Stiffness && P != Prec::F64) {
    // bricks in FP32: a lane pair per element, 2 * BLOCK lanes for a tile of BLOCK elements
    // (in FP64 the pair kernel sits at the register limit and was slower on 1M bricks)
    auto kern = k_pass1_pair<P, 2 * BLOCK>;
    if (!set_lds(kern, p.lds1)) return KB_EHIP;
    kern<<<(unsigned)p.ntiles, 2 * BLOCK, p.lds1, s>>>(m->conn, (const double4*)(ws + p.o_coords4), m->coef, p.nel,
                                                       p.nn, p.tau, p.s1, p.nb, (const uint32_t*)(ws + p.o_hist),
                                                       (uint16_t*)(ws + p.o_row1), (uint32_t*)(ws + p.o_col1),
                                                       (V*)(ws + p.o_val1), (uint32_t*)(ws + p.o_emax), status);
    KB_LAUNCH_CHECK();
    return KB_OK;
  }
  if constexpr (NEN == 8 && !FROM_VALUES && P == Prec::F64) {
    // bricks in FP64: two tiles per workgroup (two waves per SIMD while integrating)
    auto kern = k_pass1_two<NEN, P, BLOCK, OP>;
    if (!set_lds(kern, p.lds1)) return KB_EHIP;
    kern<<<(unsigned)div_up(p.ntiles, 2), 2 * BLOCK, p.lds1, s>>>(
        m->conn, (const double4*)(ws + p.o_coords4), m->coef, p.nel, p.nn, p.tau, p.s1, p.nb, p.ntiles,
        (const uint32_t*)(ws + p.o_hist), (uint16_t*)(ws + p.o_row1), (uint32_t*)(ws + p.o_col1),
        (V*)(ws + p.o_val1), (uint32_t*)(ws + p.o_emax), status);
    KB_LAUNCH_CHECK();
    return KB_OK;
  }
  auto kern = [] {
    if constexpr (NEN == 4)
      return k_pass1_tet<P, FROM_VALUES, BLOCK, OP>;
    else
      return k_pass1<NEN, P, FROM_VALUES, BLOCK, OP>;
  }();
  if (!set_lds(kern, p.lds1)) return KB_EHIP;
  // tetrahedra: persistent, the workgroups that fit on the device at once (LDS-bound),
  // at least one per XCD slot (b % 8) that owns tiles; bricks: one tile per workgroup
  const int per_cu = std::max(1, (int)(163840 / std::max<size_t>(p.lds1, 1)));
  const int64_t g1 =
      NEN == 8 ? p.ntiles
               : std::min<int64_t>(p.ntiles, std::max<int64_t>(8, (int64_t)p.cus * std::min(per_cu, 2048 / BLOCK)));
  kern<<<(unsigned)g1, BLOCK, p.lds1, s>>>(m->conn, (const double4*)(ws + p.o_coords4), m->coef, (const V*)klow, p.nel,
                                           p.nn, p.tau, p.s1, p.nb, p.ntiles, (const uint32_t*)(ws + p.o_hist),
                                           (uint16_t*)(ws + p.o_row1), (uint32_t*)(ws + p.o_col1),
                                           (V*)(ws + p.o_val1), (uint32_t*)(ws + p.o_emax), status);
  KB_LAUNCH_CHECK();
  return KB_OK;
}

// pass-1 tile sizes (elements = lanes per workgroup): {small, default} per element and
// value size; the staging LDS is tile * pairs * (8 + value bytes)
template <int NEN, Prec P>
struct TileSizes {
  static constexpr int big = NEN == 4 ? (P == Prec::F64 ? 768 : 1024) : 256;
  static constexpr int mid = NEN == 8 && P == Prec::F64 ? 192 : 0;  // FP64, many buckets
  static constexpr int small = big / 2 >= 64 && (big / 2) % 64 == 0 ? big / 2 : 64 * ((big / 2 + 63) / 64);
};

// elements of more than 8 rows: `tile` elements on kWideThreads threads, one tile per workgroup
template <int NEN, typename V>
int launch_pass1_wide(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, uint32_t* status,
                      hipStream_t s) {
  auto kern = k_pass1_wide<NEN, V>;
  if (!set_lds(kern, p.lds1)) return KB_EHIP;
  kern<<<(unsigned)p.ntiles, kWideThreads, p.lds1, s>>>(m->conn, (const V*)klow, p.nel, p.nn, p.tile, p.s1, p.nb,
                                              (const uint32_t*)(ws + p.o_hist), (uint16_t*)(ws + p.o_row1),
                                              (uint32_t*)(ws + p.o_col1), (V*)(ws + p.o_val1),
                                              (uint32_t*)(ws + p.o_emax), status);
  KB_LAUNCH_CHECK();
  return KB_OK;
}

// OP: the integrand of pass 1 when the values are not given
template <int NEN, Prec P, bool FROM_VALUES, Op OP = Op::Stiffness>
int launch_pass1(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, uint32_t* status,
                 hipStream_t s) {
  if constexpr (NEN > 8) {
    static_assert(FROM_VALUES, "elements of more than 8 rows are assembled from given values");
    return launch_pass1_wide<NEN, typename PrecTraits<P>::V>(p, m, klow, ws, status, s);
  } else {
    if (p.tile == TileSizes<NEN, P>::big)
      return launch_pass1_block<NEN, P, FROM_VALUES, TileSizes<NEN, P>::big, OP>(p, m, klow, ws, status, s);
    if (p.tile == TileSizes<NEN, P>::small)
      return launch_pass1_block<NEN, P, FROM_VALUES, TileSizes<NEN, P>::small, OP>(p, m, klow, ws, status, s);
    if constexpr (TileSizes<NEN, P>::mid > 0) {
      if (p.tile == TileSizes<NEN, P>::mid)
        return launch_pass1_block<NEN, P, FROM_VALUES, TileSizes<NEN, P>::mid, OP>(p, m, klow, ws, status, s);
    }
    return KB_EINVAL;
  }
}

// Running sums of a grouped build: read back as a second source of pairs (in), and the
// pass's entries written with their residuals and rows (out).
struct Carry {
  bool first = true;              // first pass: the status words are initialised
  const int32_t* rows = nullptr;  // in: rows, columns, values, residuals of the entries
  const int32_t* cols = nullptr;
  const void* vals = nullptr;
  const void* res = nullptr;
  const int64_t* nnz = nullptr;   // in: number of entries (device); nullptr: no input
  void* res_out = nullptr;        // out: residuals and rows of the pass's entries
  int32_t* rows_out = nullptr;
};

// pass 3, then the sub-buckets it could not hold (k_pass3_heavy: a small grid whose
// workgroups return at once when there are none)
template <typename V, bool RES>
int launch_pass3(const Plan& p, uint32_t* key2, V* val2, uint32_t* sbb, uint32_t* emax, int32_t* tcol, V* tval,
                 V* tres, uint32_t* rowoff, uint32_t* usub, uint32_t* ov_list, uint32_t* hvy, hipStream_t s) {
  const unsigned g3 = (unsigned)p.nsub;
  uint32_t* ov_count = emax + 1;
  switch (p.ht) {
    case 512:
      k_pass3<V, 512, RES><<<g3, 256, (size_t)12 << p.s2, s>>>(key2, val2, sbb, p.s2, p.colbits, p.nn, emax, tcol, tval, tres, rowoff,
                                              usub, ov_list, ov_count);
      break;
    case 1024:
      k_pass3<V, 1024, RES><<<g3, 256, (size_t)12 << p.s2, s>>>(key2, val2, sbb, p.s2, p.colbits, p.nn, emax, tcol, tval, tres,
                                               rowoff, usub, ov_list, ov_count);
      break;
    case 2048:
      k_pass3<V, 2048, RES><<<g3, 256, (size_t)12 << p.s2, s>>>(key2, val2, sbb, p.s2, p.colbits, p.nn, emax, tcol, tval, tres,
                                               rowoff, usub, ov_list, ov_count);
      break;
    default:
      k_pass3<V, 4096, RES><<<g3, 256, (size_t)12 << p.s2, s>>>(key2, val2, sbb, p.s2, p.colbits, p.nn, emax, tcol, tval, tres,
                                               rowoff, usub, ov_list, ov_count);
      break;
  }
  KB_LAUNCH_CHECK();
  auto kh = k_pass3_heavy<V, RES>;
  if (!set_lds(kh, HeavySmem::bytes())) return KB_EHIP;
  const unsigned gh = (unsigned)std::min<int64_t>(p.nsub, kHeavyGrid);
  kh<<<gh, kHeavyThreads, HeavySmem::bytes(), s>>>(key2, val2, (uint32_t*)tcol, tval, sbb, p.s2, p.colbits, p.nn, emax,
                                                   tres, rowoff, usub, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  // up to kHeavyPar of them split by many workgroups, their big leaves summed by many
  // workgroups, their first-level ranges reduced by one workgroup per compute unit, then
  // their entry counts scanned (all return at once when there are none)
  const unsigned gsplit = (unsigned)std::max(1, 2 * p.cus);
  k_heavy_rows<<<gsplit, kHeavyThreads, 0, s>>>(key2, sbb, p.colbits, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  k_heavy_layout<<<(unsigned)kHeavyPar, kHvyRows, 0, s>>>(sbb, p.colbits, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  k_heavy_hist<<<gsplit, kHeavyThreads, 0, s>>>(key2, sbb, p.colbits, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  k_heavy_starts<<<(unsigned)kHeavyPar, kHeavyThreads, 0, s>>>(sbb, p.colbits, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  k_heavy_scatter<V><<<gsplit, kHeavyThreads, 0, s>>>(key2, val2, (uint32_t*)tcol, tval, sbb, p.colbits, ov_list,
                                                      ov_count, hvy);
  KB_LAUNCH_CHECK();
  auto kl = k_heavy_bigleaf<V>;
  if (!set_lds(kl, HeavySmem::bytes())) return KB_EHIP;
  kl<<<(unsigned)std::max(1, p.cus), kHeavyThreads, HeavySmem::bytes(), s>>>((uint32_t*)tcol, tval, emax, ov_count,
                                                                           hvy);
  KB_LAUNCH_CHECK();
  auto kr = k_pass3_heavy_ranges<V, RES>;
  if (!set_lds(kr, HeavySmem::bytes())) return KB_EHIP;
  kr<<<(unsigned)std::max(1, p.cus), kHeavyThreads, HeavySmem::bytes(), s>>>(key2, val2, (uint32_t*)tcol, tval,
                                                                           p.colbits, emax, tres, ov_count, hvy);
  KB_LAUNCH_CHECK();
  k_pass3_heavy_finish<V, RES><<<(unsigned)kHeavyPar, kFinishThreads, 0, s>>>((uint32_t*)tcol, tval, tres, sbb, p.s2,
                                                                            p.nn, rowoff, usub, ov_list, ov_count, hvy);
  KB_LAUNCH_CHECK();
  return KB_OK;
}

template <typename V>
int assemble_tail(const Plan& p, unsigned char* ws, int32_t* row_ptr, int32_t* col_idx, V* vals, int64_t cap,
                  int64_t* nnz_dev, uint32_t* status, Events& ev, hipStream_t s, const Carry* cr) {
  auto* bstart = (uint32_t*)(ws + p.o_bstart);
  auto* segbase = (uint32_t*)(ws + p.o_segbase);
  auto* hist2 = (uint32_t*)(ws + p.o_hist2);
  auto* seg2b = (uint32_t*)(ws + p.o_seg2b);
  auto* emax = (uint32_t*)(ws + p.o_emax);
  auto* row1 = (uint16_t*)(ws + p.o_row1);
  auto* col1 = (uint32_t*)(ws + p.o_col1);
  auto* val1 = (V*)(ws + p.o_val1);
  auto* key2 = (uint32_t*)(ws + p.o_key2);
  auto* val2 = (V*)(ws + p.o_val2);
  auto* sbb = (uint32_t*)(ws + p.o_sbb);
  auto* rowoff = (uint32_t*)(ws + p.o_rowoff);
  auto* usub = (uint32_t*)(ws + p.o_usub);
  auto* ubase = (uint32_t*)(ws + p.o_ubase);
  auto* part = (int32_t*)(ws + p.o_part);
  // pass-3 output reuses the pass-1 buffers (dead after pass 2)
  auto* tcol = (int32_t*)col1;
  auto* tval = val1;
  KB_TRY(ev.rec(KB_STAGE_HISTOGRAM));
  if (p.nb > 0) {
    const unsigned gs = (unsigned)p.nseg_max;
    k_seg_map<<<(unsigned)p.nb, 256, 0, s>>>(segbase, seg2b);
    KB_LAUNCH_CHECK();
    if (p.seg == kSegLong)
      k_hist2<kSegLong><<<gs, 256, 4 * (size_t)p.p2, s>>>(row1, bstart, segbase, seg2b, p.nb, p.s2, p.p2, hist2);
    else
      k_hist2<kSeg><<<gs, 256, 4 * (size_t)p.p2, s>>>(row1, bstart, segbase, seg2b, p.nb, p.s2, p.p2, hist2);
    KB_LAUNCH_CHECK();
    k_colscan<<<(unsigned)p.nb, 256, 0, s>>>(hist2, bstart, segbase, p.nb, p.p2, sbb);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_STAGE_PARTITION));
  if (p.nb > 0) {
    const unsigned gs = (unsigned)p.nseg_max;
    auto k2 = p.seg == kSegLong ? k_scatter2<V, kSegLong, kSegThreads> : k_scatter2<V, kSeg, kSegThreads>;
    if (!set_lds(k2, p.lds2)) return KB_EHIP;
    k2<<<gs, kSegThreads, p.lds2, s>>>(row1, col1, val1, bstart, segbase, seg2b, hist2, sbb, p.nb, p.s2, p.p2,
                                      p.colbits, key2, val2);
    KB_LAUNCH_CHECK();
  }
  auto* tres = (V*)(ws + p.o_tres);
  KB_TRY(ev.rec(KB_STAGE_REDUCE));
  if (p.nsub > 0) {
    auto* ov_list = (uint32_t*)(ws + p.o_ovl);
    auto* hvy = (uint32_t*)(ws + p.o_hvy);
    if (cr)
      KB_TRY((launch_pass3<V, true>(p, key2, val2, sbb, emax, tcol, tval, tres, rowoff, usub, ov_list, hvy, s)));
    else
      KB_TRY((launch_pass3<V, false>(p, key2, val2, sbb, emax, tcol, tval, nullptr, rowoff, usub, ov_list, hvy, s)));
  }
  KB_TRY(ev.rec(KB_STAGE_COMPRESS));
  KB_TRY(scan((const int32_t*)usub, p.nsub, part, (int32_t*)ubase, nnz_dev, s));
  if (p.nsub > 0) {
    const unsigned gf = (unsigned)div_up(p.nsub, 4);
    auto* ov_list = (const uint32_t*)(ws + p.o_ovl);
    auto* hvy = (const uint32_t*)(ws + p.o_hvy);
    const uint32_t* ov_count = emax + 1;
    if (cr) {
      k_final<V, true><<<gf, 256, 0, s>>>(sbb, ubase, tcol, tval, tres, rowoff, p.s2, p.nn, p.nsub, row_ptr, col_idx,
                                          vals, (V*)cr->res_out, cr->rows_out, cap, status);
      KB_LAUNCH_CHECK();
      k_final_heavy<V, true><<<kFinalHeavyGrid, 256, 0, s>>>(sbb, ubase, tcol, tval, tres, rowoff, p.s2, p.nn, p.nsub,
                                                            ov_list, ov_count, hvy, col_idx, vals, (V*)cr->res_out,
                                                            cr->rows_out, cap);
    } else {
      k_final<V><<<gf, 256, 0, s>>>(sbb, ubase, tcol, tval, nullptr, rowoff, p.s2, p.nn, p.nsub, row_ptr, col_idx,
                                    vals, nullptr, nullptr, cap, status);
      KB_LAUNCH_CHECK();
      k_final_heavy<V><<<kFinalHeavyGrid, 256, 0, s>>>(sbb, ubase, tcol, tval, nullptr, rowoff, p.s2, p.nn, p.nsub,
                                                      ov_list, ov_count, hvy, col_idx, vals, nullptr, nullptr, cap);
    }
    KB_LAUNCH_CHECK();
  } else {
    k_scan_empty<<<1, 1, 0, s>>>(row_ptr, nullptr);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_N_STAGES));
  return KB_OK;
}

template <int NEN, Prec P>
int build_impl(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, int32_t* row_ptr,
               int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status, Events& ev,
               hipStream_t s, const Carry* cr = nullptr) {
  using V = typename PrecTraits<P>::V;
  auto* hist = (uint32_t*)(ws + p.o_hist);
  auto* csum = (uint32_t*)(ws + p.o_csum);
  auto* tot = (uint32_t*)(ws + p.o_tot);
  auto* part = (int32_t*)(ws + p.o_part);
  auto* total = (int64_t*)(ws + p.o_total);
  auto* bstart = (uint32_t*)(ws + p.o_bstart);
  auto* segbase = (uint32_t*)(ws + p.o_segbase);

  // tiles of running sums read back (grouped builds) follow the element tiles
  const int64_t ntc = (cr && cr->nnz && p.nb > 0) ? p.ntiles_csr : 0;
  const int64_t nt_all = p.ntiles + ntc;
  KB_TRY(ev.rec(KB_STAGE_INIT));
  if (!cr || cr->first) {
    k_init_status<<<1, 64, 0, s>>>(status, nnz_dev);
    KB_LAUNCH_CHECK();
  }
  k_fill_i32<<<1, 64, 0, s>>>((int32_t*)(ws + p.o_emax), 2, 0);
  KB_LAUNCH_CHECK();

  KB_TRY(ev.rec(KB_STAGE_COUNT));
  if (p.ntiles > 0) {
    // with no nodes every element has an index error: flagged, nothing counted
    const int nb = p.nb > 0 ? p.nb : 0;
    k_hist_buckets<NEN><<<(unsigned)p.ntiles, 256, 4 * (size_t)(nb > 0 ? nb : 1), s>>>(
        m->conn, p.nel, p.nn, p.tile, nb > 0 ? p.s1 : 30, nb, hist, status);
    KB_LAUNCH_CHECK();
  }
  if (ntc > 0) {
    k_hist_csr<<<(unsigned)ntc, 256, 4 * (size_t)p.nb, s>>>(cr->rows, cr->nnz, p.csr_cap, p.nn, p.s1, p.nb,
                                                            hist + p.ntiles * p.nb);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_STAGE_OFFSETS));
  if (p.nb > 0) {
    // tile offsets: column sums per chunk of tiles, their scan per bucket, bucket starts,
    // then the offsets in place (the histogram stays tile-major)
    const int64_t nchunk = div_up(nt_all, kColChunk);
    const dim3 gc((unsigned)nchunk, (unsigned)div_up(p.nb, 256));
    if (nchunk > 0) {
      k_col_chunks<<<gc, 256, 0, s>>>(hist, nt_all, p.nb, csum);
      KB_LAUNCH_CHECK();
    }
    k_col_scan<<<(unsigned)p.nb, 256, 0, s>>>(csum, nchunk, p.nb, tot);
    KB_LAUNCH_CHECK();
    KB_TRY(scan((const int32_t*)tot, p.nb, part, (int32_t*)bstart, total, s));
    if (nchunk > 0) {
      k_col_offsets<<<gc, 256, 0, s>>>(hist, csum, bstart, nt_all, p.nb);
      KB_LAUNCH_CHECK();
    }
    k_segments<<<1, 256, 0, s>>>(bstart, p.nb, p.seg, segbase);
    KB_LAUNCH_CHECK();
  }
  if (p.ntiles > 0 && p.nb > 0 && !klow && p.nn > 0) {
    k_pad_coords<<<(unsigned)std::min<int64_t>(div_up(p.nn, 256), 8192), 256, 0, s>>>(m->coords, p.nn,
                                                                                     (double4*)(ws + p.o_coords4));
    KB_LAUNCH_CHECK();
  }
  // the integrate stage is exactly one kernel (pass 1), for either integrand
  KB_TRY(ev.rec(KB_STAGE_INTEGRATE));
  if (p.ntiles > 0 && p.nb > 0) {
    if (klow) {
      KB_TRY((launch_pass1<NEN, P, true>(p, m, klow, ws, status, s)));
    } else if constexpr (NEN <= 8) {
      if (p.op == KB_OP_MASS)
        KB_TRY((launch_pass1<NEN, P, false, Op::Mass>(p, m, nullptr, ws, status, s)));
      else
        KB_TRY((launch_pass1<NEN, P, false>(p, m, nullptr, ws, status, s)));
    } else {
      return KB_EINVAL;  // several DOFs per node: values are always given
    }
  }
  if (ntc > 0) {
    const size_t lds = 2 * (size_t)kCsrTile * (8 + sizeof(V)) + 2 * 4 * (size_t)p.nb + 4 * (256 / 64 + 2);
    if (!set_lds(k_pass1_csr<V>, lds)) return KB_EHIP;
    k_pass1_csr<V><<<(unsigned)ntc, 256, lds, s>>>(cr->rows, cr->cols, (const V*)cr->vals, (const V*)cr->res, cr->nnz,
                                                   p.csr_cap, p.nn, p.s1, p.nb, hist + p.ntiles * p.nb,
                                                   (uint16_t*)(ws + p.o_row1), (uint32_t*)(ws + p.o_col1),
                                                   (V*)(ws + p.o_val1), (uint32_t*)(ws + p.o_emax));
    KB_LAUNCH_CHECK();
  }
  return assemble_tail<V>(p, ws, row_ptr, col_idx, (V*)vals, cap, nnz_dev, status, ev, s, cr);
}

template <int NEN>
int dispatch_build(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, int32_t* row_ptr,
                   int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status, Events& ev,
                   hipStream_t s, const Carry* cr = nullptr) {
  switch (p.prec) {
    case KB_FP64:
      return build_impl<NEN, Prec::F64>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s, cr);
    case KB_FP32:
      return build_impl<NEN, Prec::F32>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s, cr);
    default:
      return build_impl<NEN, Prec::F32FB>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s, cr);
  }
}

// Grouped build workspace: one pass's (the largest group plus the running sums read
// back), then the second set of running sums (CSR, residuals, rows, count) and the
// residuals and rows of the caller's set.  Passes alternate between the two sets so
// that the last one writes the caller's arrays.
struct GroupPlan {
  Plan p;
  int64_t group = 0, n_groups = 0;
  size_t o_rpB = 0, o_colB = 0, o_valB = 0, o_resB = 0, o_rowsB = 0, o_nnzB = 0, o_resA = 0, o_rowsA = 0, total = 0;
};

int make_group_plan(const kb_mesh* m, int prec, const kb_tuning* tu, int64_t group_elems, int64_t cap,
                    GroupPlan* gp) {
  if (!m || group_elems < 1 || cap < 0 || m->n_elem < 0) return KB_EINVAL;
  if (m->op != KB_OP_STIFFNESS && m->op != KB_OP_MASS) return KB_EINVAL;
  if (cap >= (int64_t)INT32_MAX) return KB_ERANGE;
  gp->group = std::min<int64_t>(group_elems, std::max<int64_t>(m->n_elem, 1));
  gp->n_groups = std::max<int64_t>(1, div_up(m->n_elem, gp->group));
  kb_mesh g = *m;
  g.n_elem = std::min<int64_t>(gp->group, m->n_elem);
  KB_TRY(make_plan(&g, prec, tu, &gp->p, 1, gp->n_groups > 1 ? cap : 0));
  size_t off = gp->p.total;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 1));
    return o;
  };
  const size_t c = gp->n_groups > 1 ? (size_t)cap : 0, vb = gp->p.vbytes;
  gp->o_rpB = take(gp->n_groups > 1 ? 4 * ((size_t)gp->p.nn + 1) : 0);
  gp->o_colB = take(4 * c);
  gp->o_valB = take(vb * c);
  gp->o_resB = take(vb * c);
  gp->o_rowsB = take(4 * c);
  gp->o_nnzB = take(8);
  gp->o_resA = take(vb * c);
  gp->o_rowsA = take(4 * c);
  gp->total = off;
  return KB_OK;
}

template <int NEN, Prec P>
int integrate_impl(const Plan& p, const kb_mesh* m, void* vals, uint32_t* status, Events& ev, hipStream_t s) {
  using V = typename PrecTraits<P>::V;
  KB_TRY(ev.rec(KB_STAGE_INIT));
  k_init_status<<<1, 64, 0, s>>>(status, nullptr);
  KB_LAUNCH_CHECK();
  for (int i = KB_STAGE_COUNT; i <= KB_STAGE_INTEGRATE; ++i) KB_TRY(ev.rec(i));
  if (p.nel > 0) {
    const int blk = std::min(p.block, 256);  // the kernel is built for at most 256 lanes
    if (p.op == KB_OP_MASS)
      k_integrate_store<NEN, P, Op::Mass><<<grid_for(p.nel, blk), blk, 0, s>>>(m->conn, m->coords, m->coef, p.nel,
                                                                              p.nn, p.tau, (V*)vals, status);
    else
      k_integrate_store<NEN, P><<<grid_for(p.nel, blk), blk, 0, s>>>(m->conn, m->coords, m->coef, p.nel, p.nn, p.tau,
                                                                    (V*)vals, status);
    KB_LAUNCH_CHECK();
  }
  for (int i = KB_STAGE_HISTOGRAM; i <= KB_N_STAGES; ++i) KB_TRY(ev.rec(i));
  return KB_OK;
}

template <int NEN>
int dispatch_integrate(const Plan& p, const kb_mesh* m, void* vals, uint32_t* status, Events& ev, hipStream_t s) {
  switch (p.prec) {
    case KB_FP64:
      return integrate_impl<NEN, Prec::F64>(p, m, vals, status, ev, s);
    case KB_FP32:
      return integrate_impl<NEN, Prec::F32>(p, m, vals, status, ev, s);
    default:
      return integrate_impl<NEN, Prec::F32FB>(p, m, vals, status, ev, s);
  }
}

// the batch as one mesh (its connectivity replaced by the shifted copy at launch)
int batch_as_mesh(const kb_batch* b, kb_mesh* m) {
  if (!b || b->n_mesh < 0) return KB_EINVAL;
  *m = kb_mesh{b->elem, KB_OP_STIFFNESS, b->n_elem, b->n_node, b->conn, b->coords, b->coef};
  return KB_OK;
}

// batch workspace: the pipeline's, then the shifted connectivity, the batch CSR row
// pointers and one flag word
struct BatchPlan {
  Plan p;
  size_t o_gconn = 0, o_uptr = 0, o_flags = 0, total = 0;
};

int make_batch_plan(const kb_batch* b, int prec, const kb_tuning* tu, BatchPlan* bp) {
  kb_mesh m;
  KB_TRY(batch_as_mesh(b, &m));
  KB_TRY(make_plan(&m, prec, tu, &bp->p));
  size_t off = bp->p.total;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 1));
    return o;
  };
  bp->o_gconn = take(4 * (size_t)bp->p.nen * (size_t)bp->p.nel);
  bp->o_uptr = take(4 * ((size_t)bp->p.nn + 1));
  bp->o_flags = take(4);
  bp->total = off;
  return KB_OK;
}

int check_mesh_ptrs(const kb_mesh* m, bool need_geometry) {
  if ((m->n_elem > 0 && !m->conn)) return KB_EINVAL;
  if (need_geometry && m->n_elem > 0 && (!m->coords || !m->coef)) return KB_EINVAL;
  return KB_OK;
}

}  // namespace

// Fixed scratch of kb_build_lower_csr_noalloc: one copy per device, resident until the
// process ends.  Host code never uses the array's name as an address: the device address
// is looked up once per device (hipGetSymbolAddress) and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[KB_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;

// device address of this device's scratch array, looked up on the first call per device
static int scratch_address(void** out) {
  static std::atomic<void*> scratch_ptr[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KB_EHIP;
  void* ptr = scratch_ptr[dev].load(std::memory_order_acquire);
  if (!ptr) {
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return KB_EHIP;
    scratch_ptr[dev].store(ptr, std::memory_order_release);
  }
  *out = ptr;
  return KB_OK;
}

extern "C" {

int kb_version(void) { return KB_VERSION; }

const char* kb_status_string(int code) {
  switch (code) {
    case KB_OK: return "ok";
    case KB_EINVAL: return "invalid argument";
    case KB_ERANGE: return "size exceeds int32 indexing";
    case KB_ENOSPC: return "workspace too small";
    case KB_EHIP: return "HIP launch failure";
    case (int)KB_F_INDEX: return "node id out of range";
    case (int)KB_F_REPEAT: return "node repeated within an element";
    case (int)KB_F_INVERTED: return "non-positive Jacobian determinant";
    case (int)KB_F_NONFINITE: return "non-finite input or value";
    case (int)KB_F_CAPACITY: return "nnz exceeds capacity";
    default: return "unknown status";
  }
}

int kb_plan(const kb_mesh* mesh, int prec, const kb_tuning* tuning, size_t* ws_bytes, int64_t* n_triplets) {
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p));
  if (ws_bytes) *ws_bytes = p.total;
  if (n_triplets) *n_triplets = p.T;
  return KB_OK;
}

// use_scratch: the library's fixed scratch array is the workspace (ws, ws_bytes ignored);
// every host check comes before the device is touched
static int build_common(const kb_mesh* mesh, int prec, const kb_tuning* tuning, const void* klow, void* ws,
                        size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev,
                        uint32_t* status_dev, void* stream, bool use_scratch = false) {
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p));
  KB_TRY(check_mesh_ptrs(mesh, klow == nullptr));
  if (!row_ptr || !nnz_dev || !status_dev || cap < 0) return KB_EINVAL;
  if (cap > 0 && (!col_idx || !vals)) return KB_EINVAL;
  if (use_scratch) {
    if (p.total > (size_t)KB_SCRATCH_BYTES) return KB_ENOSPC;
    KB_TRY(scratch_address(&ws));
    ws_bytes = (size_t)KB_SCRATCH_BYTES;
  }
  if (ws_bytes < p.total) return KB_ENOSPC;
  if (p.total > 0 && !ws) return KB_EINVAL;
  KB_TRY(device_cus(&p.cus));
  Events ev{tuning ? tuning->stage_events : nullptr, (hipStream_t)stream};
  auto* w = (unsigned char*)ws;
  auto s = (hipStream_t)stream;
  if (p.nen == 8) return dispatch_build<8>(p, mesh, klow, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
  return dispatch_build<4>(p, mesh, klow, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
}

int kb_build_lower_csr(const kb_mesh* mesh, int prec, const kb_tuning* tuning, void* ws, size_t ws_bytes,
                       int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev,
                       uint32_t* status_dev, void* stream) {
  return build_common(mesh, prec, tuning, nullptr, ws, ws_bytes, row_ptr, col_idx, vals, cap, nnz_dev, status_dev,
                      stream);
}

int kb_build_lower_csr_noalloc(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int32_t* row_ptr,
                               int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status_dev,
                               void* stream) {
  return build_common(mesh, prec, tuning, nullptr, nullptr, 0, row_ptr, col_idx, vals, cap, nnz_dev, status_dev,
                      stream, true);
}

int kb_assemble_lower_csr(const kb_mesh* mesh, int prec, const kb_tuning* tuning, const void* klow, void* ws,
                          size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                          int64_t* nnz_dev, uint32_t* status_dev, void* stream) {
  if (!mesh) return KB_EINVAL;
  if (mesh->n_elem > 0 && !klow) return KB_EINVAL;
  // klow selects the assembly-only path; a non-null marker is needed even when empty
  static const double kEmpty = 0.0;
  return build_common(mesh, prec, tuning, klow ? klow : (const void*)&kEmpty, ws, ws_bytes, row_ptr, col_idx, vals,
                      cap, nnz_dev, status_dev, stream);
}

int kb_plan_dof(const kb_mesh* mesh, int dof, int prec, const kb_tuning* tuning, size_t* ws_bytes,
                int64_t* n_triplets) {
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p, dof));
  if (ws_bytes) *ws_bytes = p.total;
  if (n_triplets) *n_triplets = p.T;
  return KB_OK;
}

int kb_assemble_lower_csr_dof(const kb_mesh* mesh, int dof, int prec, const kb_tuning* tuning, const void* klow,
                              void* ws, size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                              int64_t* nnz_dev, uint32_t* status_dev, void* stream) {
  if (dof == 1)
    return kb_assemble_lower_csr(mesh, prec, tuning, klow, ws, ws_bytes, row_ptr, col_idx, vals, cap, nnz_dev,
                                 status_dev, stream);
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p, dof));
  KB_TRY(check_mesh_ptrs(mesh, false));
  if (p.nel > 0 && !klow) return KB_EINVAL;
  if (!row_ptr || !nnz_dev || !status_dev || cap < 0) return KB_EINVAL;
  if (cap > 0 && (!col_idx || !vals)) return KB_EINVAL;
  if (ws_bytes < p.total) return KB_ENOSPC;
  if (!ws) return KB_EINVAL;
  KB_TRY(device_cus(&p.cus));
  auto* w = (unsigned char*)ws;
  auto s = (hipStream_t)stream;
  // the DOF view: elements of nen * dof rows over dof * n_node global DOFs
  kb_mesh vm = *mesh;
  vm.elem = p.nen;
  vm.n_node = p.nn;
  vm.conn = (const int32_t*)(w + p.o_dconn);
  if (p.nel > 0) {
    const int64_t n = p.nel * mesh->elem;
    k_dof_conn<<<(unsigned)std::min<int64_t>(div_up(n, 256), 65536), 256, 0, s>>>(mesh->conn, n, dof,
                                                                                   (int32_t*)(w + p.o_dconn));
    KB_LAUNCH_CHECK();
  }
  static const double kEmpty = 0.0;
  const void* kl = klow ? klow : (const void*)&kEmpty;  // selects the assembly-only path
  Events ev{tuning ? tuning->stage_events : nullptr, s};
  switch (p.nen) {
    case 8:  // tetrahedra, 2 DOFs
      return dispatch_build<8>(p, &vm, kl, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
    case 12:
      return dispatch_build<12>(p, &vm, kl, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
    case 16:
      return dispatch_build<16>(p, &vm, kl, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
    case 24:
      return dispatch_build<24>(p, &vm, kl, w, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ev, s);
    default:
      return KB_EINVAL;
  }
}

int kb_plan_grouped(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems, int64_t cap,
                    size_t* ws_bytes) {
  GroupPlan gp;
  KB_TRY(make_group_plan(mesh, prec, tuning, group_elems, cap, &gp));
  if (ws_bytes) *ws_bytes = gp.total;
  return KB_OK;
}

// One pass g of a grouped build: group g's elements (conn_g, coef_g: its n_elem rows)
// integrated and assembled together with the running sums of the passes before it.
// The two sets of running sums alternate (A = the caller's arrays, B = workspace) so
// that the last pass writes the caller's arrays.
static int grouped_pass(const GroupPlan& gp, const kb_mesh* mesh, int64_t g, const int32_t* conn_g,
                        const double* coef_g, unsigned char* w, int32_t* row_ptr, int32_t* col_idx, void* vals,
                        int64_t cap, int64_t* nnz_dev, uint32_t* status_dev, const kb_tuning* tuning, hipStream_t s) {
  Events none{nullptr, s};
  Events ev{tuning ? tuning->stage_events : nullptr, s};
  struct Set {
    int32_t* rp;
    int32_t* col;
    void* val;
    void* res;
    int32_t* rows;
    int64_t* nnz;
  };
  const Set A{row_ptr, col_idx, vals, w + gp.o_resA, (int32_t*)(w + gp.o_rowsA), nnz_dev};
  const Set B{(int32_t*)(w + gp.o_rpB), (int32_t*)(w + gp.o_colB), w + gp.o_valB, w + gp.o_resB,
              (int32_t*)(w + gp.o_rowsB), (int64_t*)(w + gp.o_nnzB)};
  kb_mesh mg = *mesh;  // this group's elements as a mesh; all nodes
  const int64_t e0 = g * gp.group;
  mg.n_elem = std::max<int64_t>(0, std::min<int64_t>(gp.group, mesh->n_elem - e0));
  mg.conn = conn_g;
  mg.coef = coef_g;
  Plan p = gp.p;
  p.nel = mg.n_elem;
  p.ntiles = div_up(p.nel, p.tile);
  const Set& out = ((gp.n_groups - 1 - g) % 2 == 0) ? A : B;
  const Set& in = (&out == &A) ? B : A;
  Carry cr;
  cr.first = g == 0;
  if (g > 0) {
    cr.rows = in.rows;
    cr.cols = in.col;
    cr.vals = in.val;
    cr.res = in.res;
    cr.nnz = in.nnz;
  }
  cr.res_out = out.res;
  cr.rows_out = out.rows;
  const Carry* crp = gp.n_groups > 1 ? &cr : nullptr;
  Events& e = g == gp.n_groups - 1 ? ev : none;
  if (p.nen == 8) return dispatch_build<8>(p, &mg, nullptr, w, out.rp, out.col, out.val, cap, out.nnz, status_dev, e, s, crp);
  return dispatch_build<4>(p, &mg, nullptr, w, out.rp, out.col, out.val, cap, out.nnz, status_dev, e, s, crp);
}

static int check_grouped_args(const GroupPlan& gp, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                              int64_t* nnz_dev, uint32_t* status_dev, void* ws, size_t ws_bytes) {
  if (!row_ptr || !nnz_dev || !status_dev) return KB_EINVAL;
  if (cap > 0 && (!col_idx || !vals)) return KB_EINVAL;
  if (ws_bytes < gp.total) return KB_ENOSPC;
  if (!ws) return KB_EINVAL;
  return KB_OK;
}

int kb_build_lower_csr_grouped(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems, void* ws,
                               size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                               int64_t* nnz_dev, uint32_t* status_dev, void* stream) {
  GroupPlan gp;
  KB_TRY(make_group_plan(mesh, prec, tuning, group_elems, cap, &gp));
  KB_TRY(check_mesh_ptrs(mesh, true));
  KB_TRY(check_grouped_args(gp, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ws, ws_bytes));
  KB_TRY(device_cus(&gp.p.cus));
  for (int64_t g = 0; g < gp.n_groups; ++g) {
    const int64_t e0 = g * gp.group;
    const int32_t* cg = mesh->n_elem > 0 ? mesh->conn + e0 * mesh->elem : nullptr;
    const double* fg = mesh->n_elem > 0 ? mesh->coef + e0 : nullptr;
    KB_TRY(grouped_pass(gp, mesh, g, cg, fg, (unsigned char*)ws, row_ptr, col_idx, vals, cap, nnz_dev, status_dev,
                        tuning, (hipStream_t)stream));
  }
  return KB_OK;
}

int kb_build_lower_csr_group_pass(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems,
                                  int64_t group, const int32_t* group_conn, const double* group_coef, void* ws,
                                  size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                                  int64_t* nnz_dev, uint32_t* status_dev, void* stream) {
  GroupPlan gp;
  KB_TRY(make_group_plan(mesh, prec, tuning, group_elems, cap, &gp));
  if (group < 0 || group >= gp.n_groups) return KB_EINVAL;
  const int64_t ng = std::max<int64_t>(0, std::min<int64_t>(gp.group, mesh->n_elem - group * gp.group));
  if (ng > 0 && (!group_conn || !group_coef || !mesh->coords)) return KB_EINVAL;
  KB_TRY(check_grouped_args(gp, row_ptr, col_idx, vals, cap, nnz_dev, status_dev, ws, ws_bytes));
  KB_TRY(device_cus(&gp.p.cus));
  return grouped_pass(gp, mesh, group, group_conn, group_coef, (unsigned char*)ws, row_ptr, col_idx, vals, cap,
                      nnz_dev, status_dev, tuning, (hipStream_t)stream);
}

int kb_plan_batched(const kb_batch* batch, int prec, const kb_tuning* tuning, size_t* ws_bytes,
                    int64_t* n_triplets) {
  BatchPlan bp;
  KB_TRY(make_batch_plan(batch, prec, tuning, &bp));
  if (ws_bytes) *ws_bytes = bp.total;
  if (n_triplets) *n_triplets = bp.p.T;
  return KB_OK;
}

int kb_build_lower_csr_batched(const kb_batch* batch, int prec, const kb_tuning* tuning, void* ws, size_t ws_bytes,
                               int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_off,
                               uint32_t* status_dev, void* stream) {
  BatchPlan bp;
  KB_TRY(make_batch_plan(batch, prec, tuning, &bp));
  Plan& p = bp.p;
  kb_mesh m;
  KB_TRY(batch_as_mesh(batch, &m));
  KB_TRY(check_mesh_ptrs(&m, true));
  if (!batch->elem_off || !batch->node_off || !row_ptr || !nnz_off || !status_dev || cap < 0) return KB_EINVAL;
  if (cap > 0 && (!col_idx || !vals)) return KB_EINVAL;
  if (ws_bytes < bp.total) return KB_ENOSPC;
  if (!ws) return KB_EINVAL;
  KB_TRY(device_cus(&p.cus));
  auto* w = (unsigned char*)ws;
  auto s = (hipStream_t)stream;
  auto* gconn = (int32_t*)(w + bp.o_gconn);
  auto* uptr = (int32_t*)(w + bp.o_uptr);
  auto* flags = (uint32_t*)(w + bp.o_flags);
  const int64_t nm = batch->n_mesh;
  k_fill_i32<<<1, 64, 0, s>>>((int32_t*)flags, 1, 0);
  KB_LAUNCH_CHECK();
  k_batch_check<<<grid_for(nm + 1, 256), 256, 0, s>>>(batch->elem_off, batch->node_off, nm, p.nel, p.nn, flags);
  KB_LAUNCH_CHECK();
  if (p.nel > 0 && nm > 0) {
    const unsigned g = (unsigned)std::min<int64_t>(div_up(p.nel, 256), 65536);
    if (p.nen == 8)
      k_batch_conn<8><<<g, 256, 0, s>>>(batch->conn, batch->elem_off, batch->node_off, nm, p.nel, flags, gconn);
    else
      k_batch_conn<4><<<g, 256, 0, s>>>(batch->conn, batch->elem_off, batch->node_off, nm, p.nel, flags, gconn);
    KB_LAUNCH_CHECK();
    m.conn = gconn;
  }
  // the batch's matrix: union CSR row pointers into the workspace, entries in place;
  // nnz_off[n_mesh] receives the total
  Events ev{tuning ? tuning->stage_events : nullptr, s};
  if (p.nen == 8)
    KB_TRY(dispatch_build<8>(p, &m, nullptr, w, uptr, col_idx, vals, cap, nnz_off + nm, status_dev, ev, s));
  else
    KB_TRY(dispatch_build<4>(p, &m, nullptr, w, uptr, col_idx, vals, cap, nnz_off + nm, status_dev, ev, s));
  if (nm > 0) {
    // (also with no nodes: failed offsets zero all n_node + n_mesh row pointers)
    k_batch_rows<<<(unsigned)std::min<int64_t>(div_up(p.nn + nm, 256), 65536), 256, 0, s>>>(
        uptr, batch->node_off, nm, p.nn, cap, flags, col_idx, row_ptr);
    KB_LAUNCH_CHECK();
    k_batch_meshes<<<grid_for(nm, 256), 256, 0, s>>>(uptr, batch->node_off, nm, flags, row_ptr, nnz_off, status_dev);
    KB_LAUNCH_CHECK();
  } else {
    k_batch_meshes<<<1, 64, 0, s>>>(uptr, batch->node_off, nm, flags, row_ptr, nnz_off, status_dev);
    KB_LAUNCH_CHECK();
  }
  return KB_OK;
}

// adjoint workspace: element gradients, node accumulators, one exponent word
static int adjoint_layout(const kb_mesh* m, size_t* gel, size_t* acc, size_t* emax, size_t* total) {
  if (!m) return KB_EINVAL;
  if (m->elem != KB_HEX8 && m->elem != KB_TET4) return KB_EINVAL;
  if (m->n_elem < 0 || m->n_node < 0 || m->op != KB_OP_STIFFNESS) return KB_EINVAL;
  if (m->n_node >= (int64_t)INT32_MAX || m->n_elem > (int64_t)INT32_MAX / m->elem) return KB_ERANGE;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 1));
    return o;
  };
  *gel = take(8 * 3 * (size_t)m->elem * (size_t)m->n_elem);
  *acc = take(16 * 3 * (size_t)m->n_node);
  *emax = take(4);
  *total = off;
  return KB_OK;
}

int kb_plan_adjoint(const kb_mesh* mesh, size_t* ws_bytes) {
  size_t a, b, c, t;
  KB_TRY(adjoint_layout(mesh, &a, &b, &c, &t));
  if (ws_bytes) *ws_bytes = t;
  return KB_OK;
}

int kb_adjoint_lower(const kb_mesh* mesh, const int32_t* row_ptr, const int32_t* col_idx, const double* w,
                     int64_t nnz, void* ws, size_t ws_bytes, double* grad_coef, double* grad_coords,
                     uint32_t* status_dev, void* stream) {
  size_t o_gel, o_acc, o_emax, total;
  KB_TRY(adjoint_layout(mesh, &o_gel, &o_acc, &o_emax, &total));
  KB_TRY(check_mesh_ptrs(mesh, true));
  if (!status_dev || !ws) return KB_EINVAL;
  if (ws_bytes < total) return KB_ENOSPC;
  if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return nnz < 0 ? KB_EINVAL : KB_ERANGE;
  if (mesh->n_elem > 0 && (!row_ptr || !grad_coef || (nnz > 0 && (!col_idx || !w)))) return KB_EINVAL;
  if (mesh->n_node > 0 && !grad_coords) return KB_EINVAL;
  auto s = (hipStream_t)stream;
  auto* wsb = (unsigned char*)ws;
  auto* gel = (double*)(wsb + o_gel);
  auto* acc = (unsigned long long*)(wsb + o_acc);
  auto* emax = (uint32_t*)(wsb + o_emax);
  const int64_t nel = mesh->n_elem, nn = mesh->n_node, nen = mesh->elem;
  k_init_status<<<1, 64, 0, s>>>(status_dev, nullptr);
  KB_LAUNCH_CHECK();
  k_fill_i32<<<1, 64, 0, s>>>((int32_t*)emax, 1, 0);
  KB_LAUNCH_CHECK();
  if (nn > 0) {
    k_fill_u64<<<(unsigned)std::min<int64_t>(div_up(6 * nn, 256), 65536), 256, 0, s>>>(acc, 6 * nn);
    KB_LAUNCH_CHECK();
  }
  if (nel > 0) {
    const unsigned ge = grid_for(nel, 128);
    if (nen == 8)
      k_adjoint_elems<8><<<ge, 128, 0, s>>>(mesh->conn, mesh->coords, mesh->coef, nel, nn, row_ptr, col_idx, nnz,
                                            w, grad_coef, gel, emax, status_dev);
    else
      k_adjoint_elems<4><<<ge, 128, 0, s>>>(mesh->conn, mesh->coords, mesh->coef, nel, nn, row_ptr, col_idx, nnz,
                                            w, grad_coef, gel, emax, status_dev);
    KB_LAUNCH_CHECK();
    const unsigned gs = (unsigned)div_up(nel * nen, kScatEntries);
    if (nen == 8)
      k_adjoint_scatter<8><<<gs, 256, 0, s>>>(mesh->conn, nel, nn, gel, emax, acc);
    else
      k_adjoint_scatter<4><<<gs, 256, 0, s>>>(mesh->conn, nel, nn, gel, emax, acc);
    KB_LAUNCH_CHECK();
  }
  if (nn > 0) {
    k_adjoint_nodes<<<(unsigned)std::min<int64_t>(div_up(3 * nn, 256), 65536), 256, 0, s>>>(acc, 3 * nn, emax,
                                                                                            grad_coords);
    KB_LAUNCH_CHECK();
  }
  return KB_OK;
}

int kb_integrate_lower(const kb_mesh* mesh, int prec, const kb_tuning* tuning, void* vals, uint32_t* status_dev,
                       void* stream) {
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p));
  KB_TRY(check_mesh_ptrs(mesh, true));
  if (!status_dev || (p.nel > 0 && !vals)) return KB_EINVAL;
  Events ev{tuning ? tuning->stage_events : nullptr, (hipStream_t)stream};
  auto s = (hipStream_t)stream;
  if (p.nen == 8) return dispatch_integrate<8>(p, mesh, vals, status_dev, ev, s);
  return dispatch_integrate<4>(p, mesh, vals, status_dev, ev, s);
}

}  // extern "C"
