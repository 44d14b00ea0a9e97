/*
 * kbuild.h -- C ABI of the MI355X (gfx950) builder of the lower-triangular global
 * stiffness matrix K of the 3D Poisson equation div(c grad phi) = 0.
 *
 * What is computed (Ramirez-Gil, Tsuzuki, Montealegre-Rubio, "Global finite element
 * matrix construction based on a CPU-GPU implementation"):
 *   - Eq. 6:  K = sum_e k_e  (assembly as a sum of element matrices);
 *   - Eq. 7-9: k_e = c_e * sum_q W_q |J_q| B_q^T B_q, where B = J^{-1} dN is the 3 x nen
 *     matrix of physical shape-function gradients, J = dN X (J_ij = dx_j / dxi_i) and
 *     c_e is constant per element (the paper's MP array, Section 2);
 *   - Section 3 / Alg. 2: only the lower triangle of each symmetric k_e is computed,
 *     one element per GPU lane; Alg. 1: local pairs are mapped to global indices and
 *     the triplets are summed and compressed ("sparse").
 * The global matrix is returned as lower-triangular CSR: row = max(E_a, E_b),
 * col = min(E_a, E_b); columns ascend within a row, so the diagonal is the last entry
 * of its row.  The pattern is structural: every (row, col) pair that some element
 * touches is stored, even when its value sums to zero.  Indices are 0-based int32.
 *
 * Elements and rules:
 *   KB_HEX8  8-node trilinear brick, 2x2x2 Gauss-Legendre (points +-1/sqrt(3), weights 1);
 *            local corners (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1) (1,-1,1)
 *            (1,1,1) (-1,1,1) in natural coordinates.
 *   KB_TET4  4-node linear tetrahedron, one centroid point with weight 1/6 (exact);
 *            N0 = 1-r-s-t, N1 = r, N2 = s, N3 = t.
 * Per-element lower values are packed as p = a*(a+1)/2 + b for 0 <= b <= a < nen.
 *
 * Precision modes (value type of vals / per-element outputs in parentheses):
 *   KB_FP64       all arithmetic in FP64 (double);
 *   KB_FP32       node coordinates are differenced in FP64 against the element's first
 *                 node, the rest of the integration runs in FP32; assembly sums exactly
 *                 and rounds each entry once (float).  Outside the FP32 accuracy bound
 *                 (5e-6 of sqrt(K_ii K_jj) per entry): the FP32 geometry error grows with
 *                 the Jacobian's condition number (the tests hold it to 2e-5 on
 *                 jittered meshes); KB_FP32_FB64 is the mode that meets the bound;
 *   KB_FP32_FB64  as KB_FP32, but an element whose Jacobian at some integration point
 *                 has an estimated infinity-norm condition number above tau gets its
 *                 Jacobian, determinant and inverse in FP64 (float).
 *
 * Memory and streams.  Every array passed to the kb_build / kb_integrate /
 * kb_assemble / kb_adjoint calls is a device pointer (except the kb_mesh, kb_batch
 * and kb_tuning structs themselves, which are host memory read during the call).
 * The caller owns and allocates all memory; the library allocates nothing and keeps
 * no state between calls apart from a per-device cache of the compute-unit count
 * (read once with hipDeviceGetAttribute) and, for kb_build_lower_csr_noalloc only, a
 * fixed per-device scratch array and its device address.  Work is enqueued on `stream` (a hipStream_t)
 * and the calls return without synchronising; results are valid once the stream
 * reaches that point.  Calls that share a workspace must be ordered on one stream.
 * The output of a call is bitwise deterministic for given inputs and precision.
 *
 * Errors.  Host-detectable argument errors are returned immediately (nothing is
 * enqueued).  Data errors are found on the device and OR-ed into status_dev[0]:
 * an element with an index error (KB_F_INDEX, KB_F_REPEAT) is excluded from the
 * matrix; KB_F_INVERTED and KB_F_NONFINITE elements are integrated as given.
 */
#ifndef KBUILD_H
#define KBUILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KB_VERSION 4

/* element types (value = nodes per element) */
#define KB_HEX8 8
#define KB_TET4 4

/* precision modes */
#define KB_FP64 0
#define KB_FP32 1
#define KB_FP32_FB64 2

/* return codes */
#define KB_OK 0
#define KB_EINVAL (-1)  /* null pointer, unknown element or precision, negative size  */
#define KB_ERANGE (-2)  /* n_node or n_elem * nen*(nen+1)/2 does not fit int32 indexing */
#define KB_ENOSPC (-3)  /* ws_bytes smaller than kb_plan's figure                       */
#define KB_EHIP (-4)    /* a HIP launch or event call failed                           */

/* device status words: status_dev[KB_STATUS_WORDS] (uint32) */
#define KB_STATUS_WORDS 4
/* status_dev[0]: data-error flags */
#define KB_F_INDEX 1u      /* a node id outside [0, n_node)                           */
#define KB_F_REPEAT 2u     /* a node id repeated within one element                   */
#define KB_F_INVERTED 4u   /* Jacobian determinant not > 0 at some integration point  */
#define KB_F_NONFINITE 8u  /* non-finite coordinate, coefficient or computed value    */
#define KB_F_CAPACITY 16u  /* nnz > cap: col_idx / vals were not written              */
/* status_dev[1]: number of elements integrated on the FP64 fallback (KB_FP32_FB64)
 * status_dev[2], status_dev[3]: reserved, written as 0 */

/* stages recorded into kb_tuning.stage_events (KB_N_STAGES + 1 events) */
#define KB_N_STAGES 8
#define KB_STAGE_INIT 0       /* clear status                                              */
#define KB_STAGE_COUNT 1      /* validate connectivity, pairs per row bucket per tile       */
#define KB_STAGE_OFFSETS 2    /* scan: each tile's write offset in each bucket; coordinates
                                 copied into padded 32-byte records                        */
#define KB_STAGE_INTEGRATE 3  /* integrate (or read given values), partition by bucket     */
#define KB_STAGE_HISTOGRAM 4  /* sub-bucket histogram per segment of a bucket, offsets      */
#define KB_STAGE_PARTITION 5  /* partition each bucket into sub-buckets                     */
#define KB_STAGE_REDUCE 6     /* per sub-bucket: group equal (row, col), exact sums         */
#define KB_STAGE_COMPRESS 7   /* scan of unique counts, row_ptr, col_idx / vals             */

/* element integrands (kb_mesh.op) */
#define KB_OP_STIFFNESS 0 /* k_ab = c * integral of grad N_a . grad N_b (Eq. 7-9)            */
#define KB_OP_MASS 1      /* m_ab = c * integral of N_a N_b, the consistent mass matrix
                             (Section 5): brick 2x2x2 rule, tet exact |J| (1 + delta_ab) / 120 */

typedef struct {
  int32_t elem;          /* KB_HEX8 or KB_TET4                                         */
  int32_t op;            /* KB_OP_STIFFNESS (0) or KB_OP_MASS                           */
  int64_t n_elem;        /* number of elements (>= 0)                                   */
  int64_t n_node;        /* number of nodes = matrix dimension (>= 0)                   */
  const int32_t* conn;   /* device [n_elem][nen] node ids, row-major                    */
  const double* coords;  /* device [n_node][3] x, y, z, row-major                       */
  const double* coef;    /* device [n_elem] coefficient c of each element               */
} kb_mesh;

/* Optional tuning knobs; pass NULL for defaults.  Zero fields mean "default". */
typedef struct {
  int32_t block;           /* threads per workgroup of kb_integrate_lower (64..1024,
                              at most 256 used); if it equals one of the build's
                              element tiles (tet4: 1024 / 512, FP64 768 / 384; hex8:
                              256 / 128, FP64 256 / 192 / 128) it also sets that tile,
                              which the build otherwise picks from the mesh shape
                              (FP64 hex8 256 needs at most about 2000 row buckets:
                              beyond, 192 is taken instead)                          */
  int32_t bucket_bits;     /* log2 rows per first-level bucket, <= 16 (0 = from mesh shape) */
  float fb_tau;            /* KB_FP32_FB64 condition-number threshold (> 1)             */
  int32_t sub_bits;        /* log2 rows per sub-bucket, <= bucket_bits and <= 8 (0 = auto) */
  void** stage_events;     /* NULL, or KB_N_STAGES + 1 hipEvent_t: event i is recorded
                              on the stream before stage i, the last after the final one */
  int32_t seg_pairs;       /* pairs per segment of the sub-bucket partition: 4096 or 8192
                              (0 = from the mesh shape: 8192 for tetrahedra whose short
                              segments would give fewer than 16 pairs per sub-bucket)   */
  int32_t table_slots;     /* slots of the hash table that sums one sub-bucket's pairs
                              in pass 3: 512, 1024, 2048 or 4096 (0 = about four per
                              expected distinct entry).  Fewer slots than that fit more
                              rows per sub-bucket in the same local memory; a
                              sub-bucket whose entries do not fit goes to the slower
                              overflow path, with the same result                       */
} kb_tuning;

/*
 * Size the workspace.  Host only (no device access).  On success *ws_bytes is the
 * workspace needed by kb_build_lower_csr and kb_assemble_lower_csr for this mesh
 * shape and precision, and *n_triplets = n_elem * nen*(nen+1)/2, an upper bound on
 * nnz (so cap = *n_triplets always suffices).  Either output pointer may be NULL.
 * Only elem, op, n_elem and n_node of the mesh are read.  KB_ERANGE when n_node or T
 * exceeds int32 indexing; KB_EINVAL also when the matrix has more rows than the
 * row buckets can hold: each pass-1 workgroup keeps two LDS counters per bucket of at
 * most 2^16 rows beside its staged pairs, and a sub-bucket key packs the row within its
 * sub-bucket beside a column index in 31 bits.  Without bucket_bits / sub_bits the plan
 * widens the buckets (and the sub-buckets) and narrows the element tile as the rows
 * grow: up to about 1.3e8 rows (2^27; about 7e7 for element matrices of more than 8
 * rows), where the lower pattern of a brick mesh nears the 2^31 entries of int32 indexing.
 */
int kb_plan(const kb_mesh* mesh, int prec, const kb_tuning* tuning, size_t* ws_bytes, int64_t* n_triplets);

/*
 * Full construction (Alg. 1 with the integration of Alg. 2): integrate the lower
 * triangle of every element matrix and assemble lower-triangular CSR K.
 *   ws        device workspace of ws_bytes >= kb_plan's figure (contents scratch)
 *   row_ptr   device [n_node + 1]; always written unless an argument error is returned
 *   col_idx   device [cap], vals device [cap] of double (KB_FP64) or float (otherwise);
 *             written only if nnz <= cap, else KB_F_CAPACITY is set
 *   nnz_dev   device int64, receives nnz
 *   status_dev device uint32[KB_STATUS_WORDS], overwritten (see above)
 *   stream    hipStream_t (NULL = default stream)
 * A node may be shared by any number of elements.  Rows whose entries or pairs
 * overflow the reduction's local tables (a hub node's row) are reduced on a separate
 * path that spreads them over the device, with the same exact sums and so the same bits.
 */
int kb_build_lower_csr(const kb_mesh* mesh, int prec, const kb_tuning* tuning, void* ws, size_t ws_bytes,
                       int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev,
                       uint32_t* status_dev, void* stream);

/*
 * kb_build_lower_csr without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a fixed array of KB_SCRATCH_BYTES inside the
 * library: one copy per device, held from the library's first use on that device until
 * the process ends.  The call allocates nothing (no hipMalloc, no allocating library
 * routine); its first call on a device looks up that device's copy of the array.
 *   Arguments, outputs and errors as for kb_build_lower_csr (without ws / ws_bytes);
 *   KB_ENOSPC when kb_plan's workspace figure for this mesh exceeds KB_SCRATCH_BYTES
 *   (about 3e6 lower pairs in FP32: e.g. 300,000 tetrahedra or 80,000 bricks), KB_EHIP
 *   when the array's device address cannot be found.
 * Every call on one device uses that device's single array: calls that overlap on one
 * device (other streams, other host threads) race and corrupt each other's results, so
 * the caller orders them (one stream, or events).  The array keeps the last call's
 * contents; the build initialises every part of it that it reads.
 */
#define KB_SCRATCH_BYTES (64u << 20)
int kb_build_lower_csr_noalloc(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int32_t* row_ptr,
                               int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_dev, uint32_t* status_dev,
                               void* stream);

/*
 * Integration only (Alg. 2): vals device [n_elem][nen*(nen+1)/2] of double (KB_FP64)
 * or float, element-major, packed lower order.  Elements with index errors get zeros.
 * No workspace.  status_dev as above.
 */
int kb_integrate_lower(const kb_mesh* mesh, int prec, const kb_tuning* tuning, void* vals, uint32_t* status_dev,
                       void* stream);

/*
 * Assembly only (Eq. 6 and the "sparse" step of Alg. 1) from given per-element lower
 * values klow (device [n_elem][nen*(nen+1)/2], double for KB_FP64, float otherwise);
 * mesh->coords and mesh->coef are not read and may be NULL.  Outputs as for
 * kb_build_lower_csr.  KB_FP32 and KB_FP32_FB64 behave alike here.
 */
int kb_assemble_lower_csr(const kb_mesh* mesh, int prec, const kb_tuning* tuning, const void* klow, void* ws,
                          size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                          int64_t* nnz_dev, uint32_t* status_dev, void* stream);

/*
 * Several degrees of freedom per node (Alg. 1, the mapping of local to global indices
 * with DOFs per node): element matrices of nd = nen * dof rows, local row a*dof + i
 * standing for component i of corner a, global DOF dof * E_a + i.  K has dof * n_node
 * rows.  Assembly only, from given values (as kb_assemble_lower_csr): the integrands of
 * this library are scalar, vector problems bring their own element matrices.
 *   dof       1, 2 or 3 (1 is exactly kb_assemble_lower_csr)
 *   klow      device [n_elem][nd*(nd+1)/2], packed lower order p = r*(r+1)/2 + s, s <= r,
 *             double for KB_FP64, float otherwise
 *   row_ptr   device [dof * n_node + 1]; other outputs as for kb_build_lower_csr
 * mesh->op, mesh->coords and mesh->coef are not read, nor tuning->block (the element
 * tile follows from the pairs per element).  A node id outside [0, n_node)
 * or repeated within an element is flagged as in kb_build_lower_csr and the element left
 * out.  Host only: kb_plan_dof sizes the workspace (and T = n_elem * nd*(nd+1)/2).
 * Errors: KB_EINVAL for dof outside 1..3 or a bad argument, KB_ERANGE when dof * n_node
 * or T exceeds int32 indexing, KB_ENOSPC for a short workspace.
 */
int kb_plan_dof(const kb_mesh* mesh, int dof, int prec, const kb_tuning* tuning, size_t* ws_bytes,
                int64_t* n_triplets);
int kb_assemble_lower_csr_dof(const kb_mesh* mesh, int dof, int prec, const kb_tuning* tuning, const void* klow,
                              void* ws, size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                              int64_t* nnz_dev, uint32_t* status_dev, void* stream);

/*
 * Grouped build (Eq. 10: K as the sum of the matrices of element groups, each group
 * assembled while the next is integrated).  Elements [g*G, (g+1)*G) form group g; one
 * pass per group integrates the group and, in the same pass, reads back the sums of
 * the groups before it (a lower CSR carried in the output arrays and the workspace) as
 * pairs beside the group's own, so the sums grow group by group and the last pass
 * leaves K in the outputs.  Each carried entry is held as its rounded value plus the
 * rounded residual (together about twice the value type's precision).  Each pass
 * truncates its values at its own fixed-point scale (2^-94 of its largest value), so
 * the result can differ from a single-pass build only where that truncation matters:
 * within one rounding of an entry, or a few units of 2^-94 of the largest entry
 * (measured: most meshes bit for bit; tiny entries of meshes with a wide coefficient
 * range may differ in the last bit).  One pass's pairs are
 * G * nen*(nen+1)/2 + 2 * cap, which must stay below 2^31: grouping builds meshes whose
 * n_elem * nen*(nen+1)/2 exceeds what one pass indexes, as long as nnz stays below 2^31.
 *   group_elems  G >= 1 (G >= n_elem: a single pass, as kb_build_lower_csr)
 *   cap          capacity of col_idx / vals and of the carried sums: at least the final
 *                nnz (the sums only grow), else KB_F_CAPACITY and the result is void
 *   other arguments as for kb_build_lower_csr (both operators; status accumulates over
 *   the groups; stage events, if given, time the last group's pass)
 * kb_plan_grouped sizes the workspace (host only).  Errors: KB_EINVAL (group_elems < 1,
 * a bad argument), KB_ERANGE (a pass's pairs or cap beyond int32 indexing), KB_ENOSPC.
 */
int kb_plan_grouped(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems, int64_t cap,
                    size_t* ws_bytes);
int kb_build_lower_csr_grouped(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems, void* ws,
                               size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                               int64_t* nnz_dev, uint32_t* status_dev, void* stream);

/*
 * One pass of a grouped build, for callers that stream the element groups in (Eq. 10
 * groups of a mesh whose connectivity and coefficients stay in host memory: the paper
 * uploads only the data of the group being integrated, Section 3).  Calling it for
 * group = 0, 1, ..., n_groups - 1 (n_groups = ceil(n_elem / group_elems)), in order on
 * one stream with one workspace, gives exactly what kb_build_lower_csr_grouped gives.
 *   mesh         the whole mesh: elem, op, n_elem, n_node and coords (device, all
 *                nodes) are read; conn and coef are not (may be NULL)
 *   group_conn   device [G_g][nen]: the connectivity of elements [group * group_elems,
 *                group * group_elems + G_g), G_g = min(group_elems, n_elem - group *
 *                group_elems); group_coef device [G_g] their coefficients.  Only read
 *                by the work this call enqueues: the caller may refill them once the
 *                stream has passed it (an event recorded after the call).
 *   other arguments as for kb_build_lower_csr_grouped (the same workspace and outputs
 *   on every pass; the outputs hold K after the last pass).
 * Errors as for kb_build_lower_csr_grouped; KB_EINVAL also for a group outside
 * [0, n_groups) or a null group array for a non-empty group.
 */
int kb_build_lower_csr_group_pass(const kb_mesh* mesh, int prec, const kb_tuning* tuning, int64_t group_elems,
                                  int64_t group, const int32_t* group_conn, const double* group_coef, void* ws,
                                  size_t ws_bytes, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap,
                                  int64_t* nnz_dev, uint32_t* status_dev, void* stream);

/*
 * Batches.  Many independent meshes of one element type, built by one enqueued sequence
 * of kernels (no host synchronisation, so the whole call can be captured in a HIP graph).
 * The meshes are packed back to back: mesh m owns elements [elem_off[m], elem_off[m+1])
 * and nodes [node_off[m], node_off[m+1]); its connectivity holds node ids local to the
 * mesh (0 .. node_off[m+1] - node_off[m] - 1).  No element couples two meshes, so the
 * batch's K is block diagonal and each mesh's lower CSR is what kb_build_lower_csr
 * gives for that mesh alone.  (Section 3, Eq. 10 splits one large mesh into element
 * groups integrated one after another; a batch is the converse case, many meshes too
 * small to fill the device, and is built in a single pass.)
 */
typedef struct {
  int32_t elem;             /* KB_HEX8 or KB_TET4, for every mesh                          */
  int32_t n_mesh;           /* number of meshes (>= 0)                                    */
  int64_t n_elem;           /* total elements                                             */
  int64_t n_node;           /* total nodes                                                */
  const int64_t* elem_off;  /* device [n_mesh + 1]: 0, ..., n_elem (non-decreasing)          */
  const int64_t* node_off;  /* device [n_mesh + 1]: 0, ..., n_node (non-decreasing)          */
  const int32_t* conn;      /* device [n_elem][nen], node ids local to each mesh           */
  const double* coords;     /* device [n_node][3]                                          */
  const double* coef;       /* device [n_elem]                                             */
} kb_batch;

/* Workspace and triplet bound for a batch (host only; reads elem, n_mesh, n_elem,
 * n_node).  Returns as kb_plan; T and n_node are the batch totals. */
int kb_plan_batched(const kb_batch* batch, int prec, const kb_tuning* tuning, size_t* ws_bytes,
                    int64_t* n_triplets);

/*
 * Build every mesh of a batch.  Outputs (device):
 *   row_ptr  [n_node + n_mesh]: mesh m's row pointers (node_off[m+1] - node_off[m] + 1
 *            entries, the first 0) start at row_ptr[node_off[m] + m];
 *   col_idx, vals [cap]: mesh m's entries, mesh-local column ids, start at nnz_off[m];
 *   nnz_off  int64 [n_mesh + 1]: nnz_off[n_mesh] = total nnz;
 *   status_dev as for kb_build_lower_csr; offsets that do not start at 0, decrease or
 *            do not end at the totals, and local ids outside their mesh, set KB_F_INDEX.
 * If the total nnz exceeds cap, KB_F_CAPACITY is set and col_idx / vals are not
 * written (row_ptr and nnz_off still are).  Workspace from kb_plan_batched.
 */
int kb_build_lower_csr_batched(const kb_batch* batch, int prec, const kb_tuning* tuning, void* ws, size_t ws_bytes,
                               int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t cap, int64_t* nnz_off,
                               uint32_t* status_dev, void* stream);

/*
 * Adjoint (not part of the paper; derived from Eq. 7-9).  For the loss
 * L = sum over the lower pattern of w_ij K_ij, with w (device double [nnz]) laid out
 * like the values of the lower CSR (row_ptr [n_node + 1], col_idx [nnz]) that
 * kb_build_lower_csr produced for this mesh, writes
 *   grad_coef   device double [n_elem]     dL/dc_e,
 *   grad_coords device double [n_node][3]  dL/dX (x, y, z of each node).
 * nnz is the number of entries of col_idx and w: no entry outside [0, nnz) is read,
 * and a row whose pointers fall outside it counts as missing from the pattern.
 * All arithmetic is FP64 whatever precision built K.  Node gradients are summed exactly
 * (fixed-point integers), so the output is bitwise deterministic; exact while no node
 * belongs to more than 65,536 elements.  A node pair of an element that is missing
 * from the pattern sets KB_F_INDEX (its weight is taken as 0); elements with index
 * errors contribute nothing.  An element whose Jacobian determinant is not > 0 at some
 * integration point sets KB_F_INVERTED; one whose gradients are not finite (degenerate
 * geometry, non-finite coordinates or coefficient) sets KB_F_NONFINITE, and its
 * non-finite node contributions are left out of the sums.  Workspace from
 * kb_plan_adjoint (host only).  Errors: KB_EINVAL (bad argument, nnz < 0), KB_ERANGE
 * (nnz beyond int32 indexing).
 */
int kb_plan_adjoint(const kb_mesh* mesh, size_t* ws_bytes);
int kb_adjoint_lower(const kb_mesh* mesh, const int32_t* row_ptr, const int32_t* col_idx, const double* w,
                     int64_t nnz, void* ws, size_t ws_bytes, double* grad_coef, double* grad_coords,
                     uint32_t* status_dev, void* stream);

/* Static text for a return code (negative) or a single status flag bit (positive). */
const char* kb_status_string(int code);

/* KB_VERSION of the loaded library. */
int kb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KBUILD_H */
