/*
 * mbddc.h - C ABI of the MI355X BDDC-preconditioned GMRES library.
 *
 * The library solves the Newton tangent systems of finite-element elasticity
 * (Barnafi, Pavarino, Scacchi, arXiv 2208.06191, §2 eq. "tangent problem")
 * with GMRES preconditioned by two-level BDDC (§3.2, "BDDC preconditioner").
 * The operator is given unassembled, element by element, together with a
 * non-overlapping element partition (§3.2, Omega = U Omega_i; §4, MATIS
 * storage) and a choice of primal constraints (vertices / edge averages /
 * face averages, §3.2 and §6.2).
 *
 * Conventions shared by every entry point
 *  - Every function returns MBDDC_OK (0) or a negative status; nothing throws
 *    across the ABI. mbddc_strerror() names a status.
 *  - DOF numbering is 3*node + component (the strided block-size-3 layout of
 *    §4). Vectors are "full DOF vectors" of length 3*n_nodes (summed over the
 *    instances of a batch, in instance order); clamped (Dirichlet) entries are
 *    ignored on input and written as 0 on output.
 *  - Host pointers are read during the call only and never retained. Device
 *    pointers (flag on_device = 1) must live on the handle's device and stay
 *    valid for the duration of the call.
 *  - A handle is not thread-safe; distinct handles are independent. All GPU
 *    work is enqueued on the handle's HIP stream; every call returns after the
 *    work it enqueued has completed.
 *  - Call order: create -> setup_symbolic -> set_tangent -> factor ->
 *    solve / apply / matvec (any number) ; set_tangent again replaces the
 *    operator, and solves then reuse the factors of the last factor call
 *    (lagged preconditioner) until factor is called again. Calls out of
 *    order return MBDDC_ERR_STATE.
 */
#ifndef MBDDC_H
#define MBDDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MBDDC_OK = 0,
  MBDDC_ERR_ARG = -1,        /* invalid argument (NULL, out of range, NaN in an input) */
  MBDDC_ERR_OOM = -2,        /* device allocation failed; nothing partial is kept */
  MBDDC_ERR_SINGULAR = -3,   /* zero pivot: info / mbddc_last_bad_subdomain names it (-1: coarse) */
  MBDDC_ERR_NOCONV = -4,     /* GMRES hit max_it; x holds the last iterate */
  MBDDC_ERR_DEVICE = -5,     /* a HIP runtime call failed */
  MBDDC_ERR_STATE = -6,      /* call out of order */
  MBDDC_ERR_UNSUPPORTED = -7 /* size or option outside what this build handles */
};

enum { MBDDC_HEX8 = 1, MBDDC_HEX27 = 2 };              /* Q1, Q2 hexahedra (§2) */
enum { MBDDC_PRIMAL_V = 1, MBDDC_PRIMAL_E = 2, MBDDC_PRIMAL_F = 4 }; /* §6.2 primal spaces */
/* Precision policy. Global vectors, the assembled operator, the coarse problem
 * and GMRES are FP64 in every mode. MBDDC_FP64: local factorisations and the
 * per-iteration local operators in FP64. MBDDC_MIXED: local factorisations in
 * FP64; the local operators are stored in FP32 (half the bytes each apply reads)
 * and every product with them accumulates in FP64. MBDDC_MIXED_F32FACT: local
 * factorisations in FP32 too (symmetric path: blocks of any size, the large ones
 * swept on the FP32 matrix cores with FP32 accumulation; general path: blocks up
 * to 512 rows). The FP32 local inverses are less accurate: the outer FP64 GMRES
 * absorbs the difference at the cost of iterations that depend on the problem
 * (none on the ventricle-like shell, 3 to 5 on small Q1 boxes), so this mode is
 * not held to MBDDC_MIXED's oracle + 2 iteration contract. */
enum { MBDDC_FP64 = 0, MBDDC_MIXED = 1, MBDDC_MIXED_F32FACT = 2 };
/* interface scaling of the averaging operator (mbddc_options.scaling) */
enum { MBDDC_SCALING_COUNTING = 0, MBDDC_SCALING_DELUXE = 1 };

typedef struct mbddc_ctx mbddc_ctx;

/* One mesh and its partition (§3.2). Element-local node order is lexicographic:
 * local index a + (p+1) b + (p+1)^2 c for reference-cube position (a, b, c),
 * p = 1 (HEX8) or 2 (HEX27). */
typedef struct {
  int32_t n_nodes;
  const double* coords;          /* [n_nodes*3], may be NULL (not used by the box rule) */
  int32_t n_elems;
  int32_t elem_type;             /* MBDDC_HEX8 or MBDDC_HEX27 */
  const int32_t* elem_nodes;     /* [n_elems*npe] node ids */
  int32_t n_sub;
  const int32_t* elem_part;      /* [n_elems] subdomain id in [0, n_sub) */
  const uint32_t* node_tags;     /* [n_nodes] boundary-surface bitmask, may be NULL */
  int32_t n_dirichlet;
  const int32_t* dirichlet_dofs; /* [n_dirichlet] clamped DOF ids (homogeneous) */
} mbddc_mesh;

typedef struct {
  uint32_t primal;               /* MBDDC_PRIMAL_* bitmask */
  int32_t levels;                /* 2: exact (dense FP64) coarse solve; 3: the coarse problem is itself
                                    solved approximately by one BDDC application (multilevel BDDC,
                                    §3.2 last paragraph), whose level-3 coarse problem is exact */
  int32_t coarse_group;          /* levels = 3: fine subdomain i of an instance belongs to level-2
                                    subdomain i / coarse_group (§7 uses groups of 8) */
  int32_t precision;             /* MBDDC_FP64, MBDDC_MIXED or MBDDC_MIXED_F32FACT */
  int32_t restart;               /* GMRES restart length, 1..64 */
  double rtol;                   /* relative residual target on ||b - K x||_2 */
  int32_t max_it;                /* Arnoldi steps summed over restarts */
  int32_t symmetric_hint;        /* 1: the tangent is symmetric (hyperelastic tangents): local and
                                    coarse inverses by pivot-free symmetric sweeps, which need the
                                    pivots (Schur complements of leading blocks) nonsingular: SPD
                                    local problems, coarse problems SPD or mildly indefinite;
                                    0: general path with partial pivoting (the paper's symmetry
                                    flag, §4 and §6.1) */
  const char* tune_table;        /* path of a tuning table written by mbddc_autotune (read during
                                    mbddc_setup_symbolic; MBDDC_ERR_ARG if unreadable or malformed),
                                    or NULL for the built-in choices */
  int32_t keep_coarse_matrix;    /* 1: keep S_PiPi for mbddc_get_coarse_matrix (8 n_c^2 bytes) */
  uint32_t coarse_primal;        /* levels = 3: primal globs of the level-2 decomposition
                                    (MBDDC_PRIMAL_* bitmask; default V|E|F). Level-2 nodes are the
                                    fine primal globs (three coarse components each; a component
                                    without a coarse DOF is treated as clamped), level-2 elements
                                    the fine subdomains with their matrices Phi_i^T A^(i) Phi_i;
                                    level-2 globs use the fine glob's first-node boundary tags.
                                    Level 2 and 3 are always computed in FP64. */
  int32_t graph_apply;           /* 1 (default): GMRES replays the preconditioner application (every
                                    phase, all levels) as an instantiated HIP graph captured on the
                                    handle's stream at the first iteration for each right-hand-side
                                    width; recaptured when the handle's apply buffers move. Applies
                                    whose families are being profiled run eagerly. 0: eager launches */
  int32_t packed_sym;            /* symmetric path (symmetric_hint = 1): store the symmetric blocks of the
                                    interior and interface operators (K_II^-1, D S~ D) once, as lower
                                    column panels of 256 columns, and read every stored tile once per
                                    application for both its product and its transposed product (about
                                    half their bytes for blocks of many panels). 1 (default): when that
                                    cuts the operator bytes by 10 % or more; 2: always; 0: never */
  int32_t nonsym_coarse;         /* general path (symmetric_hint = 0): 1 (default) the non-symmetric BDDC
                                    formulation (§8: a tangent whose symmetry is broken, e.g. by a
                                    follower pressure): the coarse right-hand side uses the left coarse
                                    basis Psi of the transposed constrained problems (N_i^T [Psi; L'] =
                                    [0; I]), so that the preconditioner of K^T is the transpose of that of
                                    K; the coarse matrix Psi^T K Phi equals Phi^T K Phi's formula -Lambda.
                                    0: Psi = Phi. Identical for symmetric tangents. */
  int32_t nnsp;                  /* 1: near-null-space primals (§4: the rigid motions given to BDDC as
                                    primal degrees of freedom): on every primal edge and face the
                                    constraint rows are an orthonormal basis of the six rigid motions
                                    restricted to the glob's free DOFs (candidates: translations x, y, z,
                                    then rotations about x, y, z through the glob's node centroid;
                                    modified Gram-Schmidt with one re-orthogonalisation; a candidate
                                    left with at most 1e-8 of its norm is dropped: a straight edge keeps
                                    5 rows, a planar face 6); vertices keep their component rows. Needs
                                    node coordinates (MBDDC_ERR_ARG without); levels = 3 returns
                                    MBDDC_ERR_UNSUPPORTED. 0 (default): component averages */
  int32_t scaling;               /* interface weights of the averaging operator R_D (§3.2):
                                    MBDDC_SCALING_COUNTING (default) the pseudo-inverse of the counting
                                    function; MBDDC_SCALING_DELUXE the deluxe scaling named there as the
                                    more robust option: per glob g and subdomain i the block
                                    D_g^(i) = (sum_j S_g^(j))^-1 S_g^(i) of the glob's rows and columns of
                                    the interface Schur complements, the extension averaging with D and
                                    the restriction applying D^T (computed in the factorisation, folded
                                    into the stored operators: the application costs the same).
                                    Symmetric path with FP64 local factors only (symmetric_hint = 1,
                                    precision FP64 or MIXED), else MBDDC_ERR_UNSUPPORTED; level 2 of a
                                    three-level handle keeps the counting function */
} mbddc_options;

typedef struct {
  int32_t iterations;            /* max over the systems of the call */
  int32_t restarts;
  int32_t status;
  int32_t bad_subdomain;
  double rel_res_true;           /* max over systems of ||b - K x|| / ||b|| (FP64) */
  double rel_res_est;
  double ms_setup, ms_factor, ms_solve;
  int32_t applies;               /* preconditioner applications of the call */
  int32_t applies_graphed;       /* of which replayed from a captured HIP graph */
} mbddc_info;

typedef struct {
  int64_t n_dofs;                /* 3 * total nodes */
  int64_t n_free;
  int64_t n_interface;           /* free DOFs shared by >= 2 subdomains */
  int64_t n_coarse;              /* primal constraints (all instances) */
  int64_t n_sub;
  int64_t n_instances;
  int64_t n_vertices, n_edges, n_faces;
  int64_t max_local;             /* largest local dense problem size */
  int64_t bsr_blocks;            /* 3x3 blocks of the assembled operator */
  int64_t n_sub2;                /* levels = 3: level-2 subdomains (all instances), else 0 */
  int64_t n_coarse2;             /* levels = 3: level-3 coarse DOFs (all instances), else 0 */
} mbddc_sizes;

/* Creates a handle on HIP device `hip_device`, enqueuing on `hip_stream` (a
 * hipStream_t, may be NULL for the null stream). */
int mbddc_create(mbddc_ctx** out, int hip_device, void* hip_stream);

/* Device memory provider of the handle (e.g. PyTorch's caching allocator, or a
 * serving pool): every device buffer the handle (and its level-2 instance) holds
 * is obtained by alloc(bytes, user) and returned by free_(ptr, user); blocks
 * must be device memory of the handle's device, aligned to 256 bytes (a
 * misaligned block is handed back and the allocating call fails with
 * MBDDC_ERR_ARG), and stay valid until returned. alloc returning NULL makes the
 * allocating call fail with MBDDC_ERR_OOM (nothing partial is kept). Blocks are
 * returned by mbddc_release, a new setup, buffer resizes and mbddc_destroy, each
 * after the handle's stream has finished using them. Both NULL: hipMalloc /
 * hipFree (the default). Only before the first setup (or after mbddc_release):
 * MBDDC_ERR_STATE otherwise; MBDDC_ERR_ARG if exactly one of the two is NULL. */
int mbddc_set_allocator(mbddc_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                        void (*free_)(void* ptr, void* user), void* user);

/* Returns every device buffer of the handle (through the allocator) and puts it
 * back in the created state; its streams, events and pinned host buffers are
 * kept for the next setup. */
int mbddc_release(mbddc_ctx* ctx);

/* Fills `opt` with the defaults: primal V|E, 2 levels, group 8, MIXED, restart
 * 30, rtol 1e-8, max_it 1000, level-2 primal V|E|F. */
int mbddc_default_options(mbddc_options* opt);

/* Host-side symbolic setup (§3.2 index sets: interior / interface, vertex /
 * edge / face globs, primal constraint rows, counting weights; §4 exact
 * preallocation of the assembled pattern). Copies every input. */
int mbddc_setup_symbolic(mbddc_ctx* ctx, const mbddc_mesh* mesh, const mbddc_options* opt);

/* Same for `n_inst` independent problems solved together (one launch per
 * phase for all of them); vectors and element matrices are concatenated in
 * instance order. */
int mbddc_setup_symbolic_batch(mbddc_ctx* ctx, int n_inst, const mbddc_mesh* meshes,
                               const mbddc_options* opt);

/* Device bytes the handle will hold after factor and a solve of `nrhs` (1..8)
 * right-hand sides (call after setup). */
int mbddc_footprint(const mbddc_ctx* ctx, int nrhs, size_t* device_bytes);

/* Host-only estimate (an upper bound) of the device bytes a handle set up with
 * these meshes and options holds after factor and a solve of `nrhs` (1..8)
 * right-hand sides (the admission test of the serving loop; no device is
 * touched). Same argument rules and errors as mbddc_setup_symbolic_batch. */
int mbddc_estimate_footprint(int n_inst, const mbddc_mesh* meshes, const mbddc_options* opt, int nrhs,
                             size_t* device_bytes);

int mbddc_get_sizes(const mbddc_ctx* ctx, mbddc_sizes* out);

/* Element tangents K_e, [n_elems][3npe][3npe] row-major FP64 in element-local
 * DOF order 3a + comp (all instances concatenated). Assembles the operator
 * (§3.2, A = sum_i A^(i)) on the device; keeps factors of a previous factor
 * call (lagged preconditioner). A NaN or infinite entry (found on the device,
 * before the operator is touched) returns MBDDC_ERR_ARG and leaves the handle's
 * operator and factors as they were. */
int mbddc_set_tangent(mbddc_ctx* ctx, const double* elem_K, int on_device);

/* Hyperelastic materials of the element kernels (§2): per instance, the strain energy whose
 * second Piola-Kirchhoff stress S = dPsi/dE and tangent CC = d2Psi/dE2 define the element
 * tangents. p[] holds: MBDDC_MAT_SVK (Saint Venant-Kirchhoff, Psi = lambda/2 (tr E)^2 + mu E:E,
 * the linear-elastic law written on E): lambda, mu. MBDDC_MAT_NEO_HOOKEAN (compressible,
 * Psi = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2): mu, lambda. MBDDC_MAT_GUCCIONE (§2,
 * transversely isotropic exponential law Psi = C/2 (e^Q - 1) + B/2 (J - 1) ln J with
 * Q = b_f E_ff^2 + b_t (E_ss^2 + E_nn^2 + 2 E_sn^2) + b_fs (2 E_fs^2 + 2 E_fn^2) in the fibre
 * frame (f, s, n)), with the active stress of §2, P_act = gamma (F f) (x) f / |F f|, added to
 * P: C, b_f, b_t, b_fs, B, gamma (gamma = 0: passive). Unused entries are ignored (finite). */
enum { MBDDC_MAT_SVK = 1, MBDDC_MAT_NEO_HOOKEAN = 2, MBDDC_MAT_GUCCIONE = 3 };
typedef struct {
  int32_t kind;
  double p[6];
} mbddc_material;

/* Sets the material of every instance (mats[n_instances]) for the element kernels. Needs the
 * node coordinates of every mesh (mbddc_mesh.coords at setup; MBDDC_ERR_ARG otherwise).
 * frames: [n_elems][3][3] row-major, rows the fibre, sheet and sheet-normal unit vectors of each
 * element (all instances concatenated; read for Guccione instances, which require it), or NULL
 * when no instance is Guccione. Copies everything to the device; state >= setup. */
int mbddc_set_material(mbddc_ctx* ctx, const mbddc_material* mats, const double* frames);

/* Boundary conditions of §2 on the element faces of tagged surfaces, for the element kernels:
 * a face (xi_d = 0 or 1 of an element's reference cube) carries condition b when all its nodes
 * carry every bit of bcs[b].tag (mbddc_mesh.node_tags), on instance bcs[b].instance (-1: all).
 * MBDDC_BC_ROBIN (the epicardial condition, stiffness and damping combined): traction
 * g = (a_perp N N^T + a_par (I - N N^T)) u with p = {a_perp, a_par}; MBDDC_BC_PRESSURE (the
 * endocardial follower pressure): g = p J F^-T N with p = {p, unused}; N the reference outward
 * normal. Each adds int g . v dS to the internal forces and its derivative to the tangent (not
 * symmetric for the pressure: solve with symmetric_hint = 0, the non-symmetric formulation).
 * Replaces earlier conditions; mbddc_set_material clears them. Needs mbddc_set_material. */
enum { MBDDC_BC_ROBIN = 1, MBDDC_BC_PRESSURE = 2 };
typedef struct {
  int32_t kind;
  uint32_t tag;
  int32_t instance;
  double p[2];
} mbddc_boundary;
int mbddc_set_boundary(mbddc_ctx* ctx, const mbddc_boundary* bcs, int n_bc);

/* The Newton tangent at displacement u (full DOF vector [n_dofs], host or device per
 * on_device), computed on the device (§2 "tangent problem"): for every element and Gauss point
 * of the tensor rule with p+1 points per direction on the reference cube, F = I + grad u,
 * K_e = sum_q w |J| grad N^T A grad N with A_iJkL = delta_ik S_JL + F_iI F_kK CC_IJKL; then the
 * operator is assembled as by mbddc_set_tangent (factors of an earlier factor call are kept).
 * With f_int != NULL the internal forces f_int = sum_e int P : grad N (P = F S; [n_dofs], 0 on
 * clamped DOFs; host or device per f_on_device) are written too. MBDDC_ERR_ARG on a
 * non-positive Jacobian (of the element map, or J = det F for the logarithmic laws) or a
 * non-finite value: the operator and factors are then left as they were, and a new tangent
 * must be set before the next mbddc_factor. Needs mbddc_set_material (MBDDC_ERR_STATE). */
int mbddc_set_displacement(mbddc_ctx* ctx, const double* u, int on_device, double* f_int, int f_on_device);

/* Copies the element matrices of the current operator ([n_elems][3npe][3npe], host or device). */
int mbddc_get_element_tangents(const mbddc_ctx* ctx, double* elem_K, int on_device);

/* Numeric BDDC setup (§3.2): local interior and constrained-Neumann problems,
 * coarse basis Phi, coarse matrix S_PiPi and its FP64 factorisation. With
 * levels = 3 S_PiPi is not factorised: the level-2 BDDC setup on the coarse
 * problem runs instead (its local problems, its coarse basis and the FP64
 * factorisation of the level-3 coarse matrix).
 * Returns MBDDC_ERR_SINGULAR on a zero pivot (mbddc_last_bad_subdomain: the
 * subdomain, -1 for the coarse problem; with levels = 3, -2 - j for level-2
 * subdomain j and -2 - n_sub2 for the level-3 coarse problem). */
int mbddc_factor(mbddc_ctx* ctx);

/* Right-preconditioned GMRES(restart) for `nrhs` right-hand sides (each
 * instance x each rhs is an independent system). b, x: [nrhs][n_dofs]. */
int mbddc_solve(mbddc_ctx* ctx, int nrhs, const double* b, double* x, int on_device,
                mbddc_info* info);

/* One preconditioner application z = M^-1 r (§3.2 block factorisation with
 * S_Gamma^-1 replaced by M^-1_BDDC). r, z: [nrhs][n_dofs]. */
int mbddc_apply(mbddc_ctx* ctx, int nrhs, const double* r, double* z, int on_device);

/* y = K x with the assembled FP64 operator (clamped rows/columns removed). */
int mbddc_matvec(mbddc_ctx* ctx, int nrhs, const double* x, double* y, int on_device);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): y = K x as mbddc_matvec with device pointers, making no
 * allocation. Its staging blocks (the interleaved copies of x and y, 8 * R * n_dofs bytes each,
 * R = 1, 2, 4 or 8 the smallest >= nrhs) live in one static device buffer of
 * MBDDC_NOALLOC_SCRATCH_BYTES per GPU, held from the first mbddc_create on that GPU until the
 * process ends. x, y: device pointers, [nrhs][n_dofs]. MBDDC_ERR_UNSUPPORTED when the two blocks
 * exceed the buffer (e.g. n_dofs * R > 1,048,576); MBDDC_ERR_STATE before a tangent is set.
 * Every call on a GPU shares that GPU's buffer: calls that overlap on one GPU (other threads,
 * other handles) race and must be serialised by the caller. */
#define MBDDC_NOALLOC_SCRATCH_BYTES (16u << 20)
int mbddc_matvec_noalloc(mbddc_ctx* ctx, int nrhs, const double* x, double* y);

/* Integer results of the symbolic setup, for inspection (host arrays):
 * node_glob [n_nodes total] glob id or -1; glob_kind [n_globs] 1/2/4;
 * coarse_glob/coarse_comp [n_coarse]. Any pointer may be NULL. */
int mbddc_get_globs(const mbddc_ctx* ctx, int32_t* node_glob, int32_t* n_globs, int32_t* glob_kind,
                    int32_t* coarse_glob, int32_t* coarse_comp);

/* The assembled coarse matrix S_PiPi of instance `inst` before factorisation,
 * [n_c][n_c] FP64 row-major (host). Available after factor when the options
 * asked to keep it (also with levels = 3, where it is the level-2 operator). */
int mbddc_get_coarse_matrix(const mbddc_ctx* ctx, int inst, double* out, int64_t n_c);

/* The assembled operator in 3x3-block CSR over nodes (host): rowptr [n_nodes+1],
 * colidx [blocks], vals [blocks*9] row-major blocks. */
int mbddc_get_bsr(const mbddc_ctx* ctx, int32_t* rowptr, int32_t* colidx, double* vals);

/* Host-only symbolic setup of one mesh (no device needed): sizes, glob
 * classification and per-subdomain counts. Output arrays may be NULL; sizes
 * first (call once with NULL arrays to learn them): node_glob [n_nodes],
 * glob_kind [n_globs = n_vertices + n_edges + n_faces], coarse_glob /
 * coarse_comp [n_coarse], sub_counts [n_sub * 3] = (interior, interface,
 * primal) DOFs per subdomain. */
int mbddc_inspect_symbolic(const mbddc_mesh* mesh, uint32_t primal, mbddc_sizes* sizes, int32_t* node_glob,
                           int32_t* glob_kind, int32_t* coarse_glob, int32_t* coarse_comp, int32_t* sub_counts);

/* Built-in kernel profiler. When bit f of `family_mask` is set, every launch of
 * kernel family f is bracketed by HIP events recorded on the handle's stream;
 * mbddc_get_profile() synchronises, returns per family the launch count, the
 * summed event time and the summed algorithmic bytes / flops of those launches
 * (operators and vectors counted once per launch), then resets the counters.
 * Families: see the names returned. `out` may hold `max_entries` records. */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double bytes;
  double flops;
} mbddc_kernel_stat;
int mbddc_set_profiling(mbddc_ctx* ctx, uint32_t family_mask);
/* Name of profiler family f (bit f of the mask), NULL past the last one. */
const char* mbddc_profile_family_name(int family);
int mbddc_get_profile(mbddc_ctx* ctx, mbddc_kernel_stat* out, int max_entries, int* n_entries);

/* Autotuner (kernel variants per size bucket, chosen on this handle's own matrices).
 * For every size bucket that occurs among the local symmetric inversions (n <= 128, <= 304,
 * <= 598, larger) each kernel variant that can take the bucket's matrices is timed by a full
 * numeric factorisation (best of two): 0 register-resident sweep (FP64, n <= 304), 1 one-
 * workgroup sweep with 16-index panels in LDS, 2 the same with 32-index panels, 3 batched
 * blocked sweep (FP64); then the number of input columns the apply stages in LDS (128, 256,
 * 512 or 1024), the column grouping of the local apply and the rows per workgroup of each
 * local apply phase A, C, F, H (256: four rows per lane, 128: two, 64: one) by timing applies of four
 * right-hand sides; FP64 factorisations
 * also time their batched GEMMs on the vector units (0) and the matrix cores (1). Needs a tangent (state
 * >= set_tangent) and leaves the handle factorised with the chosen table. table_out (may be
 * NULL): JSON file
 *   {"mbddc_tune": 1, "sym_fp64": [v0, v1, v2, v3], "sym_fp32": [v0, v1, v2, v3], "apply_xchunk": C,
 *    "apply_rows": [A, C, F, H], "apply_rows2": [A, C, F, H], "apply_groups": P, "gemm_mfma": G}
 * (plus informative keys; "apply_rows" and "apply_rows2" (level-2 instance of three-level
 * handles) optional, 0 = the size that pads the row counts least; "apply_groups" optional,
 * 1 = large column groups over long ranges, 0 = small groups only, -1 (default) = large when
 * some local block has 512 columns or more; "gemm_mfma" optional, default 0),
 * to be passed as options.tune_table to later handles. A table variant
 * that cannot take some matrix (size or precision) falls back to one that can. Errors as
 * mbddc_factor; MBDDC_ERR_ARG if table_out cannot be written. */
int mbddc_autotune(mbddc_ctx* ctx, const char* table_out);
/* The handle's table: sym_fp64[4], sym_fp32[4], apply_xchunk, apply_rows[4] (rows per
 * workgroup in effect for apply phases A, C, F, H), gemm_mfma; any pointer may be NULL. */
int mbddc_get_tuning(const mbddc_ctx* ctx, int32_t* sym_fp64, int32_t* sym_fp32, int32_t* apply_xchunk,
                     int32_t* apply_rows, int32_t* gemm_mfma);

/* Subdomain of the last MBDDC_ERR_SINGULAR (-1: coarse problem; see mbddc_factor). */
int mbddc_last_bad_subdomain(const mbddc_ctx* ctx);

/* GMRES iterations of every system of the last mbddc_solve: its[inst * nrhs + k] for
 * instance inst and right-hand side k (n_entries = n_instances * nrhs; at most
 * max_entries are written). Zero before the first solve. */
int mbddc_get_iterations(const mbddc_ctx* ctx, int32_t* its, int64_t max_entries, int64_t* n_entries);

int mbddc_destroy(mbddc_ctx* ctx);

/* ---- Serving: a request loop over independent tangent solves -------------
 * Not a paper step: the production pattern around it (Newton iterations of many
 * independent problems, §2: one tangent system per Newton step). A server owns
 * `max_active` worker threads, each with its own HIP stream (default priority)
 * on `hip_device`. Requests are admitted in arrival order when a worker is free
 * and the sum of the estimated footprints (mbddc_estimate_footprint) of the
 * active requests stays within `hbm_budget` bytes; requests that arrive while
 * others run are admitted as slots and memory free up, and the kernels of all
 * active requests run concurrently on the device. A request runs its Newton
 * steps on one handle: step k sets the tangent K_k, factors it (every step, or
 * only at step 0 when `lagged`, keeping the factors resident as a lagged
 * preconditioner) and solves its right-hand sides with GMRES. Each request's
 * arithmetic is the same alone and in any mix (deterministic kernels, private
 * handle and stream). */
typedef struct mbddc_server mbddc_server;

typedef struct {
  mbddc_mesh mesh;               /* the mesh arrays are copied at submit */
  mbddc_options opt;
  int32_t n_steps;               /* Newton steps, 1..16 */
  int32_t nrhs;                  /* right-hand sides per step, 1..8 (1 for on-device Newton) */
  int32_t lagged;                /* 1: factor at step 0 only; 0: factor at every step */
  const double* elem_K;          /* [n_steps][n_elems][3npe][3npe] host; read while the request runs;
                                    NULL: on-device Newton (below) */
  const double* rhs;             /* [n_steps][nrhs][n_dofs] host; read while the request runs (unused
                                    by on-device Newton) */
  double* x;                     /* [n_steps][nrhs][n_dofs] host output, written while the request runs
                                    (on-device Newton: the iterates u_1 .. u_n_steps) */
  /* On-device Newton (elem_K == NULL; the mesh must carry coordinates): step k computes the
     tangent K(u_k) and the internal forces f_int(u_k) with the element kernels
     (mbddc_set_displacement), solves K(u_k) du = f_ext - f_int(u_k) and sets u_{k+1} = u_k + du.
     All host arrays, read while the request runs. */
  const mbddc_material* material; /* [1] */
  const double* frames;          /* [n_elems][9] for a Guccione material, else NULL */
  const double* u0;              /* [n_dofs] initial displacement */
  const double* f_ext;           /* [n_dofs] external load */
} mbddc_request;

typedef struct {
  int32_t status;                /* MBDDC_OK or the first error of the request */
  int32_t n_steps;
  int32_t iterations[16];        /* GMRES iterations per step (max over its right-hand sides) */
  double rel_res_true;           /* max over steps and right-hand sides (FP64 true residual) */
  double newton_res[16];         /* on-device Newton: ||f_ext - f_int(u_k)||_2 on the free DOFs per step */
  double t_submit_ms, t_admit_ms, t_done_ms;   /* server clock (ms since mbddc_server_create) */
  size_t footprint;              /* admitted device bytes (estimate) */
} mbddc_request_result;

/* max_active 1..64 workers; hbm_budget > 0. */
int mbddc_server_create(mbddc_server** out, int hip_device, size_t hbm_budget, int max_active);

/* Queues a request; returns immediately with its ticket (>= 0). The caller keeps
 * elem_K, rhs and x alive until mbddc_server_wait returns for the ticket.
 * MBDDC_ERR_OOM if its estimated footprint exceeds the whole budget. */
int mbddc_server_submit(mbddc_server* srv, const mbddc_request* req, int64_t* ticket);

/* Blocks until the request is done and returns its result (once per ticket). */
int mbddc_server_wait(mbddc_server* srv, int64_t ticket, mbddc_request_result* res);

/* Current queue length, active requests and admitted bytes (any pointer may be NULL). */
int mbddc_server_state(mbddc_server* srv, int32_t* queued, int32_t* active, size_t* admitted_bytes);

/* Device memory of the server. Each worker keeps one handle across requests, and
 * every handle draws its buffers from one pool owned by the server (through
 * mbddc_set_allocator): a block a request gives back is handed to a later
 * request of a size it fits (at most twice the request), so once the pool holds
 * blocks of the sizes in use, requests make no hipMalloc or hipFree. Cached free
 * blocks are released (hipFree) only when a hipMalloc fails or the pool's free
 * cache would exceed the HBM budget. Counters since mbddc_server_create: device
 * allocations and frees made by the pool, bytes in use by handles, bytes cached
 * free (any pointer may be NULL). */
int mbddc_server_pool_stats(mbddc_server* srv, int64_t* device_mallocs, int64_t* device_frees,
                            size_t* bytes_in_use, size_t* bytes_cached);

/* Finishes every queued and active request, then frees the server. */
int mbddc_server_destroy(mbddc_server* srv);

const char* mbddc_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* MBDDC_H */
