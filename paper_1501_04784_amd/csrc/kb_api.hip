// kb_api.hip -- host side of the C ABI declared in include/kbuild.h.
//
// Validates arguments, carves the caller's workspace and enqueues the kernel
// sequence on the caller's stream.  Allocates nothing and keeps no state.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "kb_kernels.hpp"
#include "kbuild.h"

namespace {

using namespace kb;

constexpr size_t kAlign = 256;
constexpr float kDefaultTau = 16.0f;
constexpr int kDefaultBlock = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  int nen = 0, te = 0, prec = 0, block = kDefaultBlock, rb = 16;
  float tau = kDefaultTau;
  int64_t nel = 0, nn = 0, T = 0;
  size_t vbytes = 8;
  // workspace offsets
  size_t o_rowcnt = 0, o_rowstart = 0, o_cursor = 0, o_uniq = 0, o_klow = 0, o_icol = 0, o_ival = 0, o_rcol = 0,
         o_rval = 0, o_part = 0, total = 0;
};

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

int make_plan(const kb_mesh* m, int prec, const kb_tuning* tu, Plan* p) {
  if (!m) return KB_EINVAL;
  if (m->elem != KB_HEX8 && m->elem != KB_TET4) return KB_EINVAL;
  if (prec != KB_FP64 && prec != KB_FP32 && prec != KB_FP32_FB64) return KB_EINVAL;
  if (m->n_elem < 0 || m->n_node < 0 || m->reserved != 0) return KB_EINVAL;
  p->nen = m->elem;
  p->te = m->elem * (m->elem + 1) / 2;
  p->prec = prec;
  p->nel = m->n_elem;
  p->nn = m->n_node;
  if (p->nn >= (int64_t)INT32_MAX) return KB_ERANGE;
  if (p->nel > (int64_t)INT32_MAX / p->te) return KB_ERANGE;
  p->T = p->nel * p->te;
  p->vbytes = prec == KB_FP64 ? 8 : 4;
  if (tu) {
    if (tu->reserved != 0) return KB_EINVAL;
    if (tu->block) {
      if (tu->block < 64 || tu->block > 1024 || (tu->block & 63)) return KB_EINVAL;
      p->block = tu->block;
    }
    if (tu->fb_tau != 0.0f) {
      if (!(tu->fb_tau > 1.0f)) return KB_EINVAL;
      p->tau = tu->fb_tau;
    }
    if (tu->rows_per_block) {
      if (tu->rows_per_block < 1 || tu->rows_per_block > 1024 || (tu->rows_per_block & (tu->rows_per_block - 1)))
        return KB_EINVAL;
      p->rb = tu->rows_per_block;
    }
  }
  if (!tu || !tu->rows_per_block) {
    // about half of the LDS capacity per row block on average
    const double avg = p->nn > 0 ? (double)p->T / (double)p->nn : 1.0;
    int rb = 1;
    while (rb < 1024 && (2.0 * rb) * avg <= 0.5 * kReduceCap) rb *= 2;
    p->rb = rb;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t nn = (size_t)p->nn, T = (size_t)p->T;
  p->o_rowcnt = take(4 * nn);
  p->o_rowstart = take(4 * (nn + 1));
  p->o_cursor = take(4 * nn);
  p->o_uniq = take(4 * nn);
  p->o_klow = take(p->vbytes * T);
  p->o_icol = take(4 * T);
  p->o_ival = take(p->vbytes * T);
  p->o_rcol = take(4 * T);
  p->o_rval = take(p->vbytes * T);
  p->o_part = take(4 * (size_t)(div_up(p->nn + 1, kScanChunk) + 1));
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

// exclusive scan in[0..n) -> out[0..n], total64 optional
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

void fill(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)div_up(n, 256);
  if (g > 4096) g = 4096;
  k_fill_i32<<<g, 256, 0, s>>>(p, n, v);
}

template <typename V>
int reduce_and_compress(const Plan& p, unsigned char* ws, int32_t* row_ptr, int32_t* col_idx, V* vals, int64_t cap,
                        int64_t* nnz_dev, uint32_t* status, Events& ev, hipStream_t s) {
  auto* rowstart = (int32_t*)(ws + p.o_rowstart);
  auto* uniq = (int32_t*)(ws + p.o_uniq);
  auto* icol = (int32_t*)(ws + p.o_icol);
  auto* ival = (V*)(ws + p.o_ival);
  auto* rcol = (int32_t*)(ws + p.o_rcol);
  auto* rval = (V*)(ws + p.o_rval);
  auto* part = (int32_t*)(ws + p.o_part);
  KB_TRY(ev.rec(KB_STAGE_REDUCE));
  if (p.nn > 0) {
    const size_t lds = (size_t)kReduceCap * (sizeof(V) + 4 + 2) + 4 * (size_t)(p.rb + 1);
    k_row_reduce<V><<<grid_for(p.nn, p.rb), kReduceThreads, lds, s>>>(rowstart, p.nn, p.rb, icol, ival, rcol, rval, uniq);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_STAGE_COMPRESS));
  KB_TRY(scan(uniq, p.nn, part, row_ptr, nnz_dev, s));
  if (p.nn > 0) {
    k_compact<V><<<grid_for(p.nn, 256), 256, 0, s>>>(rowstart, row_ptr, p.nn, rcol, rval, col_idx, vals, cap, status);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_N_STAGES));
  return KB_OK;
}

template <int NEN, Prec P>
int build_impl(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, int32_t* row_ptr,
               int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status, Events& ev,
               hipStream_t s) {
  using V = typename PrecTraits<P>::V;
  auto* rowcnt = (int32_t*)(ws + p.o_rowcnt);
  auto* rowstart = (int32_t*)(ws + p.o_rowstart);
  auto* cursor = (int32_t*)(ws + p.o_cursor);
  auto* icol = (int32_t*)(ws + p.o_icol);
  auto* ival = (V*)(ws + p.o_ival);
  auto* part = (int32_t*)(ws + p.o_part);

  KB_TRY(ev.rec(KB_STAGE_INIT));
  k_init_status<<<1, 64, 0, s>>>(status, nnz_dev);
  KB_LAUNCH_CHECK();
  fill(rowcnt, p.nn, 0, s);
  fill(cursor, p.nn, 0, s);
  KB_LAUNCH_CHECK();

  KB_TRY(ev.rec(KB_STAGE_COUNT));
  if (p.nel > 0) {
    k_count<NEN><<<grid_for(p.nel, 256), 256, 0, s>>>(m->conn, p.nel, p.nn, rowcnt, status);
    KB_LAUNCH_CHECK();
  }
  KB_TRY(ev.rec(KB_STAGE_SCAN_ROWS));
  KB_TRY(scan(rowcnt, p.nn, part, rowstart, nullptr, s));

  KB_TRY(ev.rec(KB_STAGE_INTEGRATE));
  if (p.nel > 0) {
    const unsigned g = grid_for(p.nel, p.block);
    if (!klow) {
      // element values into the workspace, then the same scatter as the assembly-only path
      V* kv = (V*)(ws + p.o_klow);
      k_integrate_store<NEN, P><<<g, p.block, 0, s>>>(m->conn, m->coords, m->coef, p.nel, p.nn, p.tau, kv, status);
      KB_LAUNCH_CHECK();
      klow = kv;
    }
    k_scatter_values<NEN, V><<<g, p.block, 0, s>>>(m->conn, (const V*)klow, p.nel, p.nn, rowstart, cursor, icol, ival,
                                                  status);
    KB_LAUNCH_CHECK();
  }
  return reduce_and_compress<V>(p, ws, row_ptr, col_idx, (V*)vals, cap, nnz_dev, status, ev, s);
}

template <int NEN>
int dispatch_build(const Plan& p, const kb_mesh* m, const void* klow, unsigned char* ws, int32_t* row_ptr,
                   int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status, Events& ev,
                   hipStream_t s) {
  switch (p.prec) {
    case KB_FP64:
      return build_impl<NEN, Prec::F64>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s);
    case KB_FP32:
      return build_impl<NEN, Prec::F32>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s);
    default:
      return build_impl<NEN, Prec::F32FB>(p, m, klow, ws, row_ptr, col_idx, vals, cap, nnz_dev, status, ev, s);
  }
}

template <int NEN, Prec P>
int integrate_impl(const Plan& p, const kb_mesh* m, void* vals, uint32_t* status, Events& ev, hipStream_t s) {
  using V = typename PrecTraits<P>::V;
  KB_TRY(ev.rec(KB_STAGE_INIT));
  k_init_status<<<1, 64, 0, s>>>(status, nullptr);
  KB_LAUNCH_CHECK();
  for (int i = KB_STAGE_COUNT; i <= KB_STAGE_INTEGRATE; ++i) KB_TRY(ev.rec(i));
  if (p.nel > 0) {
    k_integrate_store<NEN, P><<<grid_for(p.nel, p.block), p.block, 0, s>>>(m->conn, m->coords, m->coef, p.nel, p.nn,
                                                                          p.tau, (V*)vals, status);
    KB_LAUNCH_CHECK();
  }
  for (int i = KB_STAGE_REDUCE; i <= KB_N_STAGES; ++i) KB_TRY(ev.rec(i));
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

int check_mesh_ptrs(const kb_mesh* m, bool need_geometry) {
  if ((m->n_elem > 0 && !m->conn)) return KB_EINVAL;
  if (need_geometry && m->n_elem > 0 && (!m->coords || !m->coef)) return KB_EINVAL;
  return KB_OK;
}

}  // namespace

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

static int build_common(const kb_mesh* mesh, int prec, const kb_tuning* tuning, const void* klow, void* ws,
                        size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev,
                        uint32_t* status_dev, void* stream) {
  Plan p;
  KB_TRY(make_plan(mesh, prec, tuning, &p));
  KB_TRY(check_mesh_ptrs(mesh, klow == nullptr));
  if (!row_ptr || !nnz_dev || !status_dev || cap < 0) return KB_EINVAL;
  if (cap > 0 && (!col_idx || !vals)) return KB_EINVAL;
  if (ws_bytes < p.total) return KB_ENOSPC;
  if (p.total > 0 && !ws) return KB_EINVAL;
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
