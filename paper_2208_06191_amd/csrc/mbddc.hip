// MI355X BDDC-preconditioned GMRES: device memory, drivers and the C ABI.
//
// Paper: Barnafi, Pavarino, Scacchi, arXiv 2208.06191. The method (§3.2):
// non-overlapping substructuring with unassembled subdomain matrices, primal
// vertex / edge / face constraints, counting-function scaling, a coarse basis
// Phi of minimum-energy extensions and coarse matrix S_PiPi; GMRES on the
// Newton tangent (§2) preconditioned by M^-1 = U diag(A_II^-1, M^-1_BDDC) L,
// the exact block factorisation of A^-1 with the interface Schur complement
// replaced by BDDC.
//
// MI355X design: every subdomain's local problems are reduced, at factor time,
// to dense operators (K_II^-1, K_GI K_II^-1, D [N^-1]_GG D, D Phi, K_II^-1 K_IG)
// obtained by batched Gauss-Jordan inversion with partial pivoting and
// batched GEMMs; the coarse matrix is inverted explicitly in FP64. One
// preconditioner application is then five launches of column-major gemv over
// all subdomains at once plus one dense FP64 coarse product: pure HBM
// streaming with every right-hand side of the call sharing each operator read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <map>
#include <type_traits>
#include <vector>

#include "mbddc.h"
#include "plan.hpp"
#include "kernels.hpp"
#include "kernels_setup.inc"
#include "kernels_apply.inc"
#include "kernels_element.inc"

using namespace mbddc;

// Static device scratch of the no-allocation entry point (mbddc_matvec_noalloc): the staging
// blocks of the operator product live here instead of in handle buffers. Each GPU the library
// runs on holds its own copy of the array until the process ends. Host code must use the
// device address taken with hipGetSymbolAddress (per device, at handle creation), never the
// array's name, which is only a host-side stand-in.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) {                        \
      last_hip_error() = e_;                       \
      return MBDDC_ERR_DEVICE;                     \
    }                                              \
  } while (0)

hipError_t& last_hip_error() {
  static thread_local hipError_t e = hipSuccess;
  return e;
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline unsigned nblk(int64_t n, int64_t b = kBlock) { return (unsigned)((n + b - 1) / b); }

struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
};

// Kernel families timed by the built-in profiler.
enum Family {
  F_ASSEMBLE_BSR, F_ASSEMBLE_LOCAL, F_GJ_KII, F_GEMM_GH, F_GEMM_S, F_CONSTRAINTS, F_GJ_P, F_EXTRACT,
  F_COARSE_ASSEMBLE, F_COARSE_GJ_SMALL, F_COARSE_DIAG, F_COARSE_PREP, F_COARSE_GEMM, F_COARSE_ROWS,
  F_APPLY_A, F_APPLY_C, F_APPLY_E, F_APPLY_F, F_APPLY_H, F_SPMV, F_KRYLOV_DOTS, F_KRYLOV_UPDATE,
  F_KRYLOV_SMALL, F_KRYLOV_VEC, F_LEVEL2_SETUP, F_LEVEL2_APPLY, F_APPLY_WHOLE, F_ELEMENT, F_APPLY_SYMRED,
  F_APPLY_HPREP, F_DELUXE, F_COUNT
};
const char* const kFamilyName[F_COUNT] = {
  "assemble_bsr", "assemble_local", "gj_interior", "gemm_condense", "gemm_schur", "constraints", "gj_interface",
  "extract_operators", "coarse_assemble", "coarse_gj_small", "coarse_gj_diag", "coarse_gj_prep", "coarse_gj_gemm",
  "coarse_gj_rows", "apply_A_interior", "apply_C_interface", "apply_E_coarse", "apply_F_coarse_ext",
  "apply_H_average", "spmv_bsr", "krylov_dots", "krylov_update", "krylov_small", "krylov_vectors",
  "level2_setup", "apply_E_level2", "apply_whole", "element_tangents", "apply_sym_reduce", "apply_H_prep", "deluxe_scaling"};

struct Profiler {
  uint32_t mask = 0;
  struct Pending { int fam; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[F_COUNT] = {};
  double ms[F_COUNT] = {}, bytes[F_COUNT] = {}, flops[F_COUNT] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

}  // namespace

namespace mbddc {

// Largest matrix of the one-workgroup symmetric sweeps with panels of BP indices (both
// panel buffers in LDS).
template <typename T>
constexpr int sym_onewg_max(int bp = 16) { return (int)((159 * 1024) / (2 * (bp + 1) * sizeof(T))); }

// Kernels for one symmetric inversion: register-resident (FP64, n <= 304), one workgroup
// with 16- or 32-index panels in LDS, or the batched blocked sweep (FP64).
enum SymVariant { SV_REG = 0, SV_BP16 = 1, SV_BP32 = 2, SV_BLOCKED = 3, SV_COUNT = 4 };
const char* const kSymVariantName[SV_COUNT] = {"register", "lds16", "lds32", "blocked"};
// Size buckets of the tuning table: n <= 128, <= 304, <= 598, larger.
constexpr int kSymBuckets = 4;
constexpr int kSymBucketMax[kSymBuckets] = {128, 304, 598, 1 << 30};
inline int sym_bucket(int n) {
  int b = 0;
  while (b < kSymBuckets - 1 && n > kSymBucketMax[b]) ++b;
  return b;
}

// Tuning table: per precision and size bucket the inversion variant, and the number of
// input columns the apply stages in LDS at a time.
struct Tuning {
  int32_t sym[2][kSymBuckets];      // [0] FP64, [1] FP32
  int32_t xchunk;
  int32_t apply_rows[4];            // rows per workgroup of apply phases A, C, F, H (64, 128, 256; 0 = by size)
  int32_t apply_rows2[4];           // the same for the level-2 instance of three-level handles
  int32_t gemm_mfma;                // batched GEMMs on the matrix cores (1) or the vector units (0)
  int32_t apply_big;                // apply column groups: 1 large first, 0 small only, -1 by size
  Tuning() {
    gemm_mfma = 0;
    apply_big = -1;
    for (int k = 0; k < 4; ++k) apply_rows[k] = apply_rows2[k] = 0;
    const int d64[kSymBuckets] = {SV_REG, SV_REG, SV_BLOCKED, SV_BLOCKED};
    const int d32[kSymBuckets] = {SV_BP32, SV_BP32, SV_BP16, SV_BLOCKED};
    for (int b = 0; b < kSymBuckets; ++b) {
      sym[0][b] = d64[b];
      sym[1][b] = d32[b];
    }
    xchunk = kApplyChunk;
  }
};

// Whether variant v can invert every matrix of size n in the given precision.
inline bool sym_variant_ok(int v, int n, bool fp32) {
  switch (v) {
    case SV_REG: return !fp32 && n <= kSymRegMax;
    case SV_BP16: return n <= (fp32 ? sym_onewg_max<float>(16) : sym_onewg_max<double>(16));
    case SV_BP32: return n <= (fp32 ? sym_onewg_max<float>(32) : sym_onewg_max<double>(32));
    case SV_BLOCKED: return true;
    default: return false;
  }
}

// One family of symmetric inversions (K_II, S + rho C^T C or T over all subdomains),
// grouped by kernel variant. Status slots follow the descriptor order of `all`: the
// one-workgroup groups (register, lds16, lds32), then the blocked matrices (sorted by
// size, descending, so that those still active at a step form a prefix).
struct SymSet {
  std::vector<GjDesc> all;          // descriptors in status-slot order
  int64_t grp_off[SV_COUNT + 1] = {};   // [grp_off[v], grp_off[v+1]) of `all` use variant v
  int grp_maxn[SV_COUNT] = {};
  std::vector<BigSym> big;
  std::vector<int2> items;          // (matrix, lower 64-tile) of the update and finish
  std::vector<int64_t> item_off;    // [big.size() + 1]
  std::vector<GemmDesc> gd;         // U = W Dinv per matrix
  std::vector<GemmItem> gitems;
  std::vector<int64_t> gitem_off;   // [big.size() + 1]
  int64_t pbuf_elems = 0;
  GjDesc* d_all = nullptr;
  BigSym* d_big = nullptr;
  int2* d_items = nullptr;
  GemmDesc* d_gd = nullptr;
  GemmItem* d_gitems = nullptr;

  // Returns false when some matrix has no usable variant (cannot happen while the blocked
  // sweep, the last fallback, takes any size in either precision).
  bool build(const std::vector<GjDesc>& src, bool fp32, const Tuning& tune) {
    all.clear(); big.clear(); items.clear(); gd.clear(); gitems.clear();
    item_off.assign(1, 0);
    gitem_off.assign(1, 0);
    std::vector<GjDesc> grp[SV_COUNT];
    for (const GjDesc& g : src) {
      int v = tune.sym[fp32 ? 1 : 0][sym_bucket(g.n)];
      if (!sym_variant_ok(v, g.n, fp32)) {   // the table's choice cannot take this one
        v = -1;
        for (int u : {SV_REG, SV_BP32, SV_BP16, SV_BLOCKED})
          if (sym_variant_ok(u, g.n, fp32)) { v = u; break; }
        if (v < 0) return false;
      }
      grp[v].push_back(g);
    }
    std::stable_sort(grp[SV_BLOCKED].begin(), grp[SV_BLOCKED].end(),
                     [](const GjDesc& a, const GjDesc& b) { return a.n > b.n; });
    for (int v = 0; v < SV_COUNT; ++v) {
      grp_off[v] = (int64_t)all.size();
      grp_maxn[v] = 1;
      for (const GjDesc& g : grp[v]) {
        all.push_back(g);
        grp_maxn[v] = std::max(grp_maxn[v], g.n);
      }
    }
    grp_off[SV_COUNT] = (int64_t)all.size();
    pbuf_elems = 0;
    for (const GjDesc& g : grp[SV_BLOCKED]) {
      const int32_t j = (int32_t)big.size();
      BigSym b{};
      b.off = g.off; b.n = g.n; b.ld = g.ld; b.stat = (int32_t)(grp_off[SV_BLOCKED] + j); b.pw = pbuf_elems;
      pbuf_elems += 2LL * g.n * kSymCB;
      big.push_back(b);
      const int nt = (g.n + kUpdTile - 1) / kUpdTile;
      for (int t = 0; t < nt * (nt + 1) / 2; ++t) items.push_back(make_int2(j, t));
      item_off.push_back((int64_t)items.size());
      GemmDesc m{};
      m.M = g.n; m.N = kSymCB; m.K = kSymCB; m.lda = kSymCB; m.ldb = kSymCB; m.ldc = kSymCB; m.ldci = kSymCB;
      m.tiles_n = kSymCB / 64; m.alpha = 1.0; m.beta = 0.0;
      m.oA = b.pw; m.oB = (int64_t)j * kSymCB * kSymCB; m.oC = b.pw + (int64_t)g.n * kSymCB; m.oCi = 0;
      gd.push_back(m);
      for (int a = 0; a < (g.n + 63) / 64; ++a)
        for (int bb = 0; bb < m.tiles_n; ++bb) gitems.push_back({j, a, bb, 0});
      gitem_off.push_back((int64_t)gitems.size());
    }
    return true;
  }
};

}  // namespace mbddc

struct mbddc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  mbddc_options opt{};
  int state = 0;                 // 0 created, 1 symbolic, 2 tangent, 3 factored
  bool mixed = true;             // apply operators in FP32
  bool fact32 = false;           // local factorisations in FP32
  Plan plan;
  int last_bad = 0;
  size_t bytes = 0;              // device bytes currently held
  std::vector<DevMem> allocs;
  // device memory provider (mbddc_set_allocator); NULL: hipMalloc / hipFree
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  int32_t* d_flag = nullptr;     // one-word result of the input checks
  int32_t* h_flag = nullptr;     // pinned host copy of it
  std::vector<int32_t> last_its; // iterations of each (instance, rhs) system of the last solve
  int32_t last_nrhs = 0;

  // sizes
  int64_t nblocks = 0, w_elems = 0, op_elems = 0, kcl_elems = 0, piv_elems = 0, kc_elems = 0;
  int max_cols = 0, coarse_max_nc = 0;
  std::vector<SubDev> subs;
  std::vector<GjDesc> gj_kii, gj_p, gj_coarse_small;
  std::vector<int32_t> coarse_large;                 // instances inverted by the blocked path
  std::vector<GjDesc> gj_kii_large, gj_p_large;      // general path: blocks above kGjMax rows (multi-workgroup
                                                     // Gauss-Jordan, one matrix at a time)
  int32_t gen_large_max = 0;                        // largest row stride among them
  struct PivGemm { int32_t n, ld; GemmDesc* d_gd; GemmItem* d_items; int32_t n_items; };
  std::vector<PivGemm> piv_gemm;                     // rank-64 update descriptors per matrix shape
  std::vector<GemmDesc> gemm_desc;
  std::vector<GemmItem> gemm_items_gh, gemm_items_s, gemm_items_g, gemm_items_ssym, gemm_items_phi, gemm_items_stil;
  std::vector<GjDesc> gj_x;                          // (S + rho C^T C) blocks of the symmetric path
  std::vector<GjDesc> gj_t;                          // T = C X C^T blocks too large for LDS (symmetric path)
  SymSet set_kii, set_x, set_t, set_dlx;                      // symmetric path: the three inversion families
  Tuning tune;                                       // kernel variants (tuning table or defaults)
  int32_t apply_rows_eff[4] = {256, 256, 256, 256};  // rows per workgroup of apply phases A, C, F, H
  int64_t big_pbuf = 0, big_count = 0;               // batched blocked sweep: panel elements, matrices
  bool sym = false;                                  // symmetric (SPD) factor path
  std::vector<ApplyItem> itA, itC, itE, itF, itH;
  int coarse_rl = 4;                // rows per lane of the coarse product (64 RL rows per workgroup)
  std::vector<int64_t> inst_coarse_off, inst_kc_off;
  std::vector<int32_t> inst_nc, inst_kc_ld, inst_nchunk, coarse_inst, cslot_sub;
  std::vector<int32_t> chunk_inst, inst_chunk_off;
  std::vector<int64_t> chunk_begin;
  int32_t nchunk_max = 1;

  // device arrays (plan)
  SubDev* d_subs = nullptr;
  int32_t *d_sub_dofs = nullptr, *d_sub_elems = nullptr, *d_elem_npe = nullptr, *d_elem_ldof = nullptr;
  int64_t *d_ke_off = nullptr, *d_elem_ldof_off = nullptr;
  int32_t *d_cons_ptr = nullptr, *d_cons_idx = nullptr;
  double* d_cons_w = nullptr;
  int32_t *d_slot_dof = nullptr, *d_slot_ifx = nullptr, *d_ifx_ptr = nullptr, *d_ifx_slots = nullptr;
  double* d_slot_w = nullptr;
  uint8_t* d_slot_owner = nullptr;
  int32_t *d_cslot_coarse = nullptr, *d_cslot_sub = nullptr, *d_coarse_ptr = nullptr, *d_coarse_slots = nullptr,
          *d_coarse_inst = nullptr;
  int64_t *d_inst_coarse_off = nullptr, *d_inst_kc_off = nullptr;
  int32_t *d_inst_nc = nullptr, *d_inst_kc_ld = nullptr, *d_inst_nchunk = nullptr;
  int32_t *d_bsr_rowptr = nullptr, *d_bsr_col = nullptr, *d_bsr_rownode = nullptr, *d_bsr_cptr = nullptr,
          *d_bsr_kstride = nullptr;
  int64_t* d_bsr_contrib = nullptr;
  uint8_t* d_free = nullptr;
  int32_t* d_dof_inst = nullptr;
  GjDesc *d_gj_kii = nullptr, *d_gj_p = nullptr, *d_gj_cs = nullptr;
  GemmDesc* d_gemm_desc = nullptr;
  GemmItem *d_gemm_gh = nullptr, *d_gemm_s = nullptr, *d_gemm_g = nullptr, *d_gemm_ssym = nullptr,
           *d_gemm_phi = nullptr, *d_gemm_stil = nullptr;
  GjDesc* d_gj_x = nullptr;
  GjDesc* d_gj_t = nullptr;
  GemmDesc* d_csym_gd = nullptr;       // panel GEMM of the blocked coarse sweep, one per large instance
  GemmItem* d_csym_items = nullptr;
  std::vector<int64_t> csym_item_off;  // [coarse_large.size() + 1]
  double* d_rho = nullptr;
  ApplyItem *d_itA = nullptr, *d_itC = nullptr, *d_itE = nullptr, *d_itF = nullptr, *d_itH = nullptr;
  // packed symmetric phases A and C: tiles (sub, first row of the tile, first column of the panel,
  // rows), partial-product sizes (R-vectors) and buffers
  bool packed = false;
  std::vector<ApplyItem> itSA, itSC, itRA;   // itRA: phase A's tiles of G on the packed path
  ApplyItem *d_itSA = nullptr, *d_itSC = nullptr, *d_itRA = nullptr;
  std::vector<int32_t> kig_ptr, kig_col;   // K_IG rows of the packed path's phase H (SubDev::kig_*)
  int32_t *d_kig_ptr = nullptr, *d_kig_col = nullptr;
  // symmetric path: interface column groups of the sparse products G^T = K_II^-1 K_IG and
  // S = K_GG - K_GI G^T (ColGroup), their union rows, and the products' dynamic LDS
  std::vector<ColGroup> cgroups;
  std::vector<int32_t> cg_rows;
  ColGroup* d_cgroups = nullptr;
  int32_t* d_cg_rows = nullptr;
  size_t cg_lds = 16;
  // deluxe scaling: blocks per (subdomain, glob) and shared globs (DlxBlock / DlxGlob), each
  // interface slot's block and position in it, per-subdomain scratch offsets, the sweep set of
  // the summed blocks and the GEMM items of D = (sum S)^-1 S
  bool deluxe = false;
  std::vector<DlxBlock> dlx_blk;
  std::vector<DlxGlob> dlx_glob;
  std::vector<int32_t> dlx_idx, dlx_gblk, dlx_ent_blk, dlx_ent_pos;
  std::vector<int64_t> dlx_tmp_off;
  int64_t dlx_s_elems = 0, dlx_t_elems = 0, dlx_tmp_elems = 0;
  std::vector<GjDesc> gj_dlx;
  std::vector<GemmItem> gemm_items_dlx;
  DlxBlock* d_dlx_blk = nullptr;
  DlxGlob* d_dlx_glob = nullptr;
  int32_t *d_dlx_idx = nullptr, *d_dlx_gblk = nullptr, *d_dlx_ent_blk = nullptr, *d_dlx_ent_pos = nullptr;
  int64_t* d_dlx_tmp_off = nullptr;
  double *d_dlx_S = nullptr, *d_dlx_D = nullptr, *d_dlx_T = nullptr, *d_dlx_tmp = nullptr, *d_ones = nullptr;
  GemmItem* d_gemm_dlx = nullptr;
  int64_t np_total = 0, tp_total = 0;
  double *d_np = nullptr, *d_tp = nullptr, *d_cin = nullptr;
  int32_t *d_chunk_inst = nullptr, *d_inst_chunk_off = nullptr;
  int64_t* d_chunk_begin = nullptr;

  // device arrays (numeric)
  double* d_Ke = nullptr;
  double* d_vals = nullptr;
  void* d_W = nullptr;          // factor-precision work matrices
  void* d_Op = nullptr;         // apply operators
  double* d_Kcl = nullptr;      // local coarse matrices
  double* d_Kc = nullptr;       // coarse matrices, inverted in place
  double* d_Kc_keep = nullptr;  // copy of the assembled coarse matrices (optional)
  int32_t* d_piv = nullptr;
  int32_t* d_status = nullptr;  // per GJ descriptor
  int32_t* d_piv_c = nullptr;   // coarse pivots
  double *d_cDinv = nullptr, *d_cY = nullptr, *d_cCcol = nullptr;
  double* d_amax = nullptr;
  int64_t status_len = 0;
  double *d_bpanel = nullptr, *d_bdinv = nullptr, *d_bthr = nullptr;   // batched blocked sweep

  // per-call buffers (sized for R right-hand sides)
  int R_alloc = 0;
  double *d_tb = nullptr, *d_wb = nullptr, *d_cc = nullptr;
  int Y_R = 0;                   // layout (R) of the apply output block currently in d_Y
  double* d_ep = nullptr;
  double *d_X = nullptr, *d_Y = nullptr, *d_io = nullptr;
  int64_t apply_gen = 0;                 // bumped whenever the apply's buffers move
  hipStream_t cap_stream = nullptr;      // capture stream of the apply graphs (default priority)
  hipGraphExec_t apply_exec[4] = {};     // captured d_X -> d_Y applies per width R = 1, 2, 4, 8
  int64_t apply_exec_gen[4] = {};
  int32_t n_applies = 0, n_applies_graphed = 0;
  // Krylov buffers
  int R_kry = 0, restart_kry = 0;
  double *d_V = nullptr, *d_Z = nullptr, *d_Wv = nullptr, *d_B = nullptr, *d_x = nullptr, *d_r = nullptr;
  double *d_part = nullptr, *d_part2 = nullptr, *d_npart = nullptr;
  double *d_h1 = nullptr, *d_h2 = nullptr, *d_Hs = nullptr, *d_cs = nullptr, *d_sn = nullptr, *d_g = nullptr,
         *d_hnorm = nullptr, *d_y = nullptr, *d_beta = nullptr;
  int32_t *d_jsys = nullptr, *d_nk = nullptr;
  uint8_t *d_active = nullptr, *d_mode = nullptr, *d_fin = nullptr;
  // per-system GMRES state sent in one copy when the host changes it:
  // [jsys int32 x nsys][its int32 x nsys][active x nsys][mode x nsys]; d_jsys, d_its, d_active and
  // d_mode point into d_kstate
  uint8_t* d_kstate = nullptr;
  int64_t kstate_n = 0;          // systems the state buffers were sized for (>= the current count)
  int32_t* d_its = nullptr;
  double* d_bnorm = nullptr;
  uint8_t* h_kstate = nullptr;   // pinned host
  double* h_est = nullptr;       // pinned host, two slots of kstate_n (consecutive GMRES steps)
  hipEvent_t ev_step[2] = {nullptr, nullptr};
  double* h_norm = nullptr;      // pinned host
  int64_t h_cap = 0;             // systems the pinned host buffers hold
  Profiler prof;
  hipStream_t aux = nullptr;     // lookahead stream of the coarse sweep (default priority)
  hipStream_t side = nullptr;    // operator extraction overlapped with the coarse factorisation (default priority)
  hipEvent_t ev_side = nullptr;
  bool side_pending = false;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  // algorithmic bytes / flops per launch, filled by build_layout
  double op_bytes[F_COUNT] = {};
  double vec_words[F_COUNT] = {};   // FP64 vector words per right-hand side
  double fam_flops[F_COUNT] = {};
  // three levels: the coarse problem is a level-2 BDDC instance of its own (FP64)
  mbddc_ctx* child = nullptr;
  std::vector<int32_t> l2_dof;      // [n_coarse] level-2 DOF of each coarse DOF
  std::vector<int32_t> l2_eidx;     // [n_cslots] level-2 element-local DOF of each coarse slot
  int32_t* d_l2_eidx = nullptr;
  int32_t* d_l2_inv = nullptr;      // [child n_dofs] coarse DOF of each level-2 DOF, or -1
  // element kernels (mbddc_set_material / mbddc_set_displacement)
  std::vector<double> h_coords;     // [n_nodes*3] all instances, empty if some mesh came without
  bool have_material = false;
  bool ke_valid = false;            // d_Ke holds the element matrices of the current operator
  std::vector<int32_t> el_list[2];  // elements of order 1 / 2
  double* d_coords = nullptr;
  double* d_u = nullptr;
  double* d_frames = nullptr;
  double* d_fe = nullptr;
  double* d_fint = nullptr;
  int32_t* d_elem_nodes = nullptr;
  int64_t* d_elem_node_off = nullptr;
  int32_t* d_elem_mat = nullptr;
  MatDev* d_mats = nullptr;
  int32_t* d_el_list[2] = {nullptr, nullptr};
  int64_t* d_fe_off = nullptr;
  int32_t* d_ne_ptr = nullptr;
  int64_t* d_ne_ent = nullptr;
  // boundary conditions on element faces (mbddc_set_boundary)
  std::vector<uint32_t> h_tags;     // [n_nodes] all instances (zeros where a mesh came without)
  std::vector<int32_t> bc_items[2]; // per element order: (element, first face) pairs
  std::vector<int32_t> bc_end[2];
  int32_t* d_bc_items[2] = {nullptr, nullptr};
  int32_t* d_bc_end[2] = {nullptr, nullptr};
  int32_t* d_faces = nullptr;
  BcDev* d_bcs = nullptr;
};

namespace {

// A block goes back to a custom allocator only after every stream of the handle is done with
// it (the allocator may hand it to work on another stream at once; hipFree waits by itself).
void release_block(mbddc_ctx* c, void* p) {
  if (c->free_fn) {
    for (hipStream_t s : {c->stream, c->side, c->aux})
      if (s) (void)hipStreamSynchronize(s);
    if (!c->stream) (void)hipDeviceSynchronize();
    c->free_fn(p, c->alloc_user);
  } else {
    (void)hipFree(p);
  }
}

template <typename T>
int dalloc(mbddc_ctx* c, T** p, int64_t n) {
  size_t b = std::max<int64_t>(n, 1) * sizeof(T);
  b = round_up(b, 256);
  void* q = nullptr;
  if (c->alloc_fn) {
    q = c->alloc_fn(b, c->alloc_user);
    if (!q) return MBDDC_ERR_OOM;
    if ((reinterpret_cast<uintptr_t>(q) & 255) != 0) {   // the kernels assume 256-byte aligned blocks
      c->free_fn(q, c->alloc_user);
      return MBDDC_ERR_ARG;
    }
  } else {
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return MBDDC_ERR_OOM;
    }
  }
  c->allocs.push_back({q, b});
  c->bytes += b;
  *p = reinterpret_cast<T*>(q);
  return MBDDC_OK;
}

template <typename T>
void dfree(mbddc_ctx* c, T*& p) {
  if (!p) return;
  // only blocks this handle holds are released: a pointer left over from buffers already
  // released (a new setup, mbddc_release) is merely cleared
  for (size_t i = 0; i < c->allocs.size(); ++i) {
    if (c->allocs[i].p == (void*)p) {
      c->bytes -= c->allocs[i].bytes;
      c->allocs.erase(c->allocs.begin() + i);
      release_block(c, (void*)p);
      break;
    }
  }
  p = nullptr;
}

// Device buffers (and the level-2 child); the handle's streams, events and pinned host buffers
// stay, so that a handle set up again reuses them.
void free_all(mbddc_ctx* c);
void clear_pointers(mbddc_ctx* c);

void release_buffers(mbddc_ctx* c) {
  if (c->child) {   // rebuilt by every setup: torn down whole
    free_all(c->child);
    delete c->child;
    c->child = nullptr;
  }
  for (hipGraphExec_t& g : c->apply_exec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  for (auto& a : c->allocs) release_block(c, a.p);
  c->allocs.clear();
  c->bytes = 0;
  clear_pointers(c);
}

// Clears every device pointer of the handle after its buffers were released, so that no stale
// address (possibly handed out again by the allocator) is taken for a live buffer.
void clear_pointers(mbddc_ctx* c) {
  auto cl = [](auto*& p) { p = nullptr; };
  cl(c->d_B);
  cl(c->d_Hs);
  cl(c->d_Kc);
  cl(c->d_Kc_keep);
  cl(c->d_Kcl);
  cl(c->d_Ke);
  cl(c->d_V);
  cl(c->d_Wv);
  cl(c->d_X);
  cl(c->d_Y);
  cl(c->d_Z);
  cl(c->d_amax);
  cl(c->d_bdinv);
  cl(c->d_beta);
  cl(c->d_bnorm);
  cl(c->d_bpanel);
  cl(c->d_bsr_col);
  cl(c->d_bsr_contrib);
  cl(c->d_bsr_cptr);
  cl(c->d_bsr_kstride);
  cl(c->d_bsr_rownode);
  cl(c->d_bsr_rowptr);
  cl(c->d_bthr);
  cl(c->d_cCcol);
  cl(c->d_cDinv);
  cl(c->d_cY);
  cl(c->d_cc);
  cl(c->d_chunk_begin);
  cl(c->d_chunk_inst);
  cl(c->d_coarse_inst);
  cl(c->d_coarse_ptr);
  cl(c->d_coarse_slots);
  cl(c->d_cons_idx);
  cl(c->d_cons_ptr);
  cl(c->d_cons_w);
  cl(c->d_cs);
  cl(c->d_cslot_coarse);
  cl(c->d_cslot_sub);
  cl(c->d_csym_gd);
  cl(c->d_csym_items);
  cl(c->d_dof_inst);
  cl(c->d_elem_ldof);
  cl(c->d_elem_ldof_off);
  cl(c->d_elem_npe);
  cl(c->d_ep);
  cl(c->d_fin);
  cl(c->d_flag);
  cl(c->d_free);
  cl(c->d_g);
  cl(c->d_gemm_desc);
  cl(c->d_gemm_g);
  cl(c->d_gemm_gh);
  cl(c->d_gemm_phi);
  cl(c->d_gemm_s);
  cl(c->d_gemm_ssym);
  cl(c->d_gemm_stil);
  cl(c->d_gj_cs);
  cl(c->d_gj_kii);
  cl(c->d_gj_p);
  cl(c->d_gj_t);
  cl(c->d_gj_x);
  cl(c->d_h1);
  cl(c->d_h2);
  cl(c->d_hnorm);
  cl(c->d_ifx_ptr);
  cl(c->d_ifx_slots);
  cl(c->d_inst_chunk_off);
  cl(c->d_inst_coarse_off);
  cl(c->d_inst_kc_ld);
  cl(c->d_inst_kc_off);
  cl(c->d_inst_nc);
  cl(c->d_inst_nchunk);
  cl(c->d_io);
  cl(c->d_itA);
  cl(c->d_itC);
  cl(c->d_itE);
  cl(c->d_itF);
  cl(c->d_itH);
  cl(c->d_ke_off);
  cl(c->d_kstate);
  cl(c->d_l2_eidx);
  cl(c->d_l2_inv);
  cl(c->d_nk);
  cl(c->d_npart);
  cl(c->d_part);
  cl(c->d_part2);
  cl(c->d_piv);
  cl(c->d_piv_c);
  cl(c->d_r);
  cl(c->d_rho);
  cl(c->d_slot_dof);
  cl(c->d_slot_ifx);
  cl(c->d_slot_owner);
  cl(c->d_slot_w);
  cl(c->d_sn);
  cl(c->d_status);
  cl(c->d_sub_dofs);
  cl(c->d_sub_elems);
  cl(c->d_subs);
  cl(c->d_tb);
  cl(c->d_vals);
  cl(c->d_wb);
  cl(c->d_x);
  cl(c->d_y);
  cl(c->d_W);
  cl(c->d_Op);
  cl(c->d_jsys);
  cl(c->d_its);
  cl(c->d_active);
  cl(c->d_mode);
  for (SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
    cl(S->d_all); cl(S->d_big); cl(S->d_items); cl(S->d_gd); cl(S->d_gitems);
  }
  cl(c->d_coords); cl(c->d_u); cl(c->d_frames); cl(c->d_fe); cl(c->d_fint); cl(c->d_elem_nodes);
  cl(c->d_elem_node_off); cl(c->d_elem_mat); cl(c->d_mats); cl(c->d_el_list[0]); cl(c->d_el_list[1]);
  cl(c->d_fe_off); cl(c->d_ne_ptr); cl(c->d_ne_ent);
  cl(c->d_itSA); cl(c->d_itSC); cl(c->d_itRA); cl(c->d_np); cl(c->d_tp); cl(c->d_cin); cl(c->d_kig_ptr); cl(c->d_kig_col); cl(c->d_cgroups); cl(c->d_cg_rows);
  cl(c->d_dlx_blk); cl(c->d_dlx_glob); cl(c->d_dlx_idx); cl(c->d_dlx_gblk); cl(c->d_dlx_ent_blk);
  cl(c->d_dlx_ent_pos); cl(c->d_dlx_tmp_off); cl(c->d_dlx_S); cl(c->d_dlx_D); cl(c->d_dlx_T); cl(c->d_dlx_tmp);
  cl(c->d_ones); cl(c->d_gemm_dlx);
  cl(c->d_bc_items[0]); cl(c->d_bc_items[1]); cl(c->d_bc_end[0]); cl(c->d_bc_end[1]); cl(c->d_faces);
  cl(c->d_bcs);
  c->piv_gemm.clear();
  c->bc_items[0].clear(); c->bc_items[1].clear(); c->bc_end[0].clear(); c->bc_end[1].clear();
  c->have_material = false;
}

void free_all(mbddc_ctx* c) {
  if (c->child) {
    free_all(c->child);
    delete c->child;
    c->child = nullptr;
  }
  for (auto& e : c->prof.pending) {
    c->prof.pool.push_back(e.a);
    c->prof.pool.push_back(e.b);
  }
  c->prof.pending.clear();
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  c->prof.pool.clear();
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_side) (void)hipEventDestroy(c->ev_side);
  c->side = nullptr;
  c->ev_side = nullptr;
  c->side_pending = false;
  if (c->ev_a) (void)hipEventDestroy(c->ev_a);
  if (c->ev_b) (void)hipEventDestroy(c->ev_b);
  for (hipEvent_t& e : c->ev_step) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (c->aux) (void)hipStreamDestroy(c->aux);
  c->ev_a = c->ev_b = nullptr;
  c->aux = nullptr;
  release_buffers(c);
  if (c->h_est) (void)hipHostFree(c->h_est);
  if (c->h_norm) (void)hipHostFree(c->h_norm);
  if (c->h_kstate) (void)hipHostFree(c->h_kstate);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  c->h_est = c->h_norm = nullptr;
  c->h_kstate = nullptr;
  c->h_flag = nullptr;
  c->h_cap = 0;
}

template <typename T>
int upload(mbddc_ctx* c, T** p, const std::vector<T>& v) {
  int st = dalloc(c, p, (int64_t)v.size());
  if (st) return st;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return MBDDC_OK;
}

#define CHK(x)                 \
  do {                         \
    int s_ = (x);              \
    if (s_ != MBDDC_OK) return s_; \
  } while (0)

// Brackets one launch (or launch group) of family f with events on the handle's stream.
struct ProfScope {
  mbddc_ctx* c;
  int f;
  hipEvent_t a = nullptr;
  double bytes, flops;
  ProfScope(mbddc_ctx* c_, int f_, double bytes_, double flops_) : c(c_), f(f_), bytes(bytes_), flops(flops_) {
    if (c->prof.mask & (1u << f)) {
      a = c->prof.get();
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = c->prof.get();
    (void)hipEventRecord(b, c->stream);
    c->prof.pending.push_back({f, a, b});
    c->prof.launches[f]++;
    c->prof.bytes[f] += bytes;
    c->prof.flops[f] += flops;
  }
};

int apply_R(int nrhs) {
  if (nrhs <= 1) return 1;
  if (nrhs <= 2) return 2;
  if (nrhs <= 4) return 4;
  return 8;
}

size_t elem_size(bool mixed) { return mixed ? sizeof(float) : sizeof(double); }

// ----------------------------------------------------------------------------
// symbolic layout on top of the host plan
// ----------------------------------------------------------------------------
// Tuning of a level-2 instance: its parent's table, with the parent's level-2 apply rows.
Tuning child_tuning(const Tuning& t) {
  Tuning u = t;
  for (int k = 0; k < 4; ++k) u.apply_rows[k] = t.apply_rows2[k];
  u.apply_big = -1;
  return u;
}

// Structural pattern of K_IG^(i) (interior row, interface column: the pairs that share an
// element), as CSR rows over the interior appended to ptr / col; sets d.kig_ptr / d.kig_col and
// returns the entry count.
int64_t kig_pattern(const Plan& P, const SubLayout& L, std::vector<int32_t>& ptr, std::vector<int32_t>& col,
                    SubDev& d) {
  std::vector<std::vector<int32_t>> rows(L.nI);
  std::vector<int32_t> in, ifc;
  for (int32_t k = 0; k < L.n_elems; ++k) {
    const int64_t e = L.elem_off + k;
    const int32_t npe = P.elem_npe[P.sub_elems[e]];
    const int32_t* ld = P.elem_ldof.data() + P.elem_ldof_off[e];
    in.clear();
    ifc.clear();
    for (int32_t a = 0; a < 3 * npe; ++a) {
      if (ld[a] < 0) continue;
      (ld[a] < L.nI ? in : ifc).push_back(ld[a]);
    }
    if (ifc.empty()) continue;
    for (int32_t i : in)
      for (int32_t g : ifc) rows[i].push_back(g - L.nI);
  }
  d.kig_ptr = (int64_t)ptr.size();
  d.kig_col = (int64_t)col.size();
  int32_t n = 0;
  ptr.push_back(0);
  for (auto& r : rows) {
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    col.insert(col.end(), r.begin(), r.end());
    n += (int32_t)r.size();
    ptr.push_back(n);
  }
  return n;
}

// Column groups of the sparse condensation for subdomain s: kCgW consecutive interface columns
// (fewer where the union of their K_IG rows would pass kCgMaxRows) with that union.
void col_groups(const Plan& P, const SubLayout& L, int32_t s, std::vector<ColGroup>& groups,
                std::vector<int32_t>& rows_out) {
  std::vector<std::vector<int32_t>> cols(L.nG);   // interior rows coupled to each interface column
  std::vector<int32_t> in, ifc;
  for (int32_t k = 0; k < L.n_elems; ++k) {
    const int64_t e = L.elem_off + k;
    const int32_t npe = P.elem_npe[P.sub_elems[e]];
    const int32_t* ld = P.elem_ldof.data() + P.elem_ldof_off[e];
    in.clear();
    ifc.clear();
    for (int32_t a = 0; a < 3 * npe; ++a) {
      if (ld[a] < 0) continue;
      (ld[a] < L.nI ? in : ifc).push_back(ld[a]);
    }
    for (int32_t g : ifc) cols[g - L.nI].insert(cols[g - L.nI].end(), in.begin(), in.end());
  }
  for (auto& c : cols) {
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
  }
  std::vector<int32_t> u;
  for (int32_t h0 = 0; h0 < L.nG;) {
    int32_t nh = std::min<int32_t>(kCgW, L.nG - h0);
    for (;;) {
      u.clear();
      for (int32_t j = 0; j < nh; ++j) u.insert(u.end(), cols[h0 + j].begin(), cols[h0 + j].end());
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      if ((int32_t)u.size() <= kCgMaxRows || nh == 1) break;
      nh = (nh + 1) / 2;
    }
    ColGroup g{};
    g.row_off = (int64_t)rows_out.size(); g.sub = s; g.h0 = h0; g.nh = nh; g.nu = (int32_t)u.size();
    rows_out.insert(rows_out.end(), u.begin(), u.end());
    groups.push_back(g);
    h0 += nh;
  }
}

// Row blocks of the local apply phases: at most 64, 128 or 256 rows per workgroup per phase, from
// the tuning table, or (0) the one of 128 and 256 that pads the phase's row counts least (256 on ties).
void build_apply_items(mbddc_ctx* c) {
  c->itA.clear(); c->itC.clear(); c->itF.clear(); c->itH.clear();
  std::vector<ApplyItem>* lists[4] = {&c->itA, &c->itC, &c->itF, &c->itH};
  const bool gonly = c->packed;   // phase A multiplies by G alone on the packed path
  auto rows_of = [gonly](const SubDev& d, int k) -> int64_t {
    return k == 0 ? (gonly ? d.nG : d.nI + d.nG) : (k == 1 ? d.nG + d.nc : (k == 2 ? d.nG : d.nI));
  };
  for (int k = 0; k < 4; ++k) {
    int rw = c->tune.apply_rows[k];
    if (rw != 64 && rw != 128 && rw != 256) {
      int64_t pad[2] = {0, 0};
      for (const SubDev& d : c->subs)
        for (int q = 0; q < 2; ++q) {
          const int64_t w = q ? 256 : 128, r = rows_of(d, k);
          pad[q] += std::max<int64_t>(1, (r + w - 1) / w) * w - r;
        }
      rw = pad[0] < pad[1] ? 128 : 256;
    }
    c->apply_rows_eff[k] = rw;
    // a subdomain's rows split into equal blocks (multiples of 4) of at most rw rows, so that
    // the workgroups of a phase carry about the same work
    for (int64_t s = 0; s < (int64_t)c->subs.size(); ++s) {
      const int64_t r = rows_of(c->subs[s], k);
      const int64_t nb = std::max<int64_t>(1, (r + rw - 1) / rw);
      const int64_t bs = std::max<int64_t>(4, round_up((r + nb - 1) / nb, 4));
      for (int64_t b = 0; b < nb; ++b)
        lists[k]->push_back({(int32_t)s, (int32_t)(b * bs), 0, (int32_t)std::max<int64_t>(0, std::min(bs, r - b * bs))});
    }
  }
}

// Deluxe scaling layout: the glob blocks of every subdomain's interface (entries in interface
// order, i.e. ascending DOF, so that the subdomains sharing a glob list it alike), the shared
// globs with their summed blocks, and the GEMMs D_g^(i) = (sum_j S_g^(j))^-1 S_g^(i).
int build_deluxe(mbddc_ctx* c) {
  const Plan& P = c->plan;
  c->dlx_blk.clear(); c->dlx_glob.clear(); c->dlx_idx.clear(); c->dlx_gblk.clear();
  c->dlx_ent_blk.clear(); c->dlx_ent_pos.clear(); c->dlx_tmp_off.clear(); c->gj_dlx.clear();
  c->gemm_items_dlx.clear();
  c->dlx_s_elems = c->dlx_t_elems = c->dlx_tmp_elems = 0;
  if (!c->deluxe) return MBDDC_OK;
  if (!c->sym || c->fact32) return MBDDC_ERR_UNSUPPORTED;
  c->dlx_ent_blk.assign(P.n_slots, -1);
  c->dlx_ent_pos.assign(P.n_slots, -1);
  std::map<int32_t, std::vector<int32_t>> members;   // glob -> its blocks
  for (int64_t s = 0; s < P.n_sub; ++s) {
    const SubDev& d = c->subs[s];
    std::map<int32_t, std::vector<int32_t>> pos;
    for (int32_t j = 0; j < d.nG; ++j) {
      const int32_t g = P.node_glob[P.slot_dof[d.if_off + j] / 3];
      if (g < 0) return MBDDC_ERR_ARG;
      pos[g].push_back(j);
    }
    for (auto& kv : pos) {
      const int32_t id = (int32_t)c->dlx_blk.size(), n = (int32_t)kv.second.size();
      DlxBlock b{};
      b.off = c->dlx_s_elems; b.idx_off = (int64_t)c->dlx_idx.size(); b.toff = -1; b.n = n; b.sub = (int32_t)s;
      c->dlx_s_elems += (int64_t)n * n;
      for (int32_t k = 0; k < n; ++k) {
        c->dlx_idx.push_back(kv.second[k]);
        c->dlx_ent_blk[d.if_off + kv.second[k]] = id;
        c->dlx_ent_pos[d.if_off + kv.second[k]] = k;
      }
      c->dlx_blk.push_back(b);
      members[kv.first].push_back(id);
    }
    c->dlx_tmp_off.push_back(c->dlx_tmp_elems);
    c->dlx_tmp_elems += std::max<int64_t>((int64_t)d.nG * d.nG, (int64_t)d.nG * d.nc);
  }
  for (auto& kv : members) {
    DlxGlob g{};
    g.toff = c->dlx_t_elems; g.n = c->dlx_blk[kv.second[0]].n;
    g.first = (int32_t)c->dlx_gblk.size(); g.count = (int32_t)kv.second.size();
    const int32_t gid = (int32_t)c->dlx_glob.size();
    c->dlx_t_elems += (int64_t)g.n * g.n;
    for (int32_t b : kv.second) {
      if (c->dlx_blk[b].n != g.n) return MBDDC_ERR_ARG;   // a glob seen with different sizes
      c->dlx_blk[b].toff = g.toff;
      c->dlx_gblk.push_back(b);
    }
    c->dlx_glob.push_back(g);
    c->gj_dlx.push_back({g.toff, g.n, g.n, 0, gid, 0});
  }
  for (const DlxBlock& b : c->dlx_blk) {   // D = T^-1 S: A from the summed blocks, B and C the blocks
    GemmDesc gd{};
    gd.M = b.n; gd.N = b.n; gd.K = b.n; gd.lda = b.n; gd.ldb = b.n; gd.ldc = b.n; gd.ldci = b.n;
    gd.oA = b.toff; gd.oB = b.off; gd.oC = b.off; gd.oCi = b.off; gd.alpha = 1.0; gd.beta = 0.0;
    gd.tiles_n = (b.n + 63) / 64;
    const int32_t id = (int32_t)c->gemm_desc.size();
    c->gemm_desc.push_back(gd);
    for (int32_t a = 0; a < (b.n + 63) / 64; ++a)
      for (int32_t t = 0; t < gd.tiles_n; ++t) c->gemm_items_dlx.push_back({id, a, t, 0});
  }
  return MBDDC_OK;
}

int build_layout(mbddc_ctx* c) {
  const Plan& P = c->plan;
  c->subs.assign(P.n_sub, SubDev{});
  int64_t w = 0, op = 0, kcl = 0, piv = 0;
  c->gj_kii.clear();
  c->gj_p.clear();
  c->gj_kii_large.clear();
  c->gj_p_large.clear();
  c->gen_large_max = 0;
  c->piv_gemm.clear();
  c->gemm_desc.clear();
  c->gemm_items_gh.clear();
  c->gemm_items_s.clear();
  c->gemm_items_g.clear();
  c->gemm_items_ssym.clear();
  c->gemm_items_phi.clear();
  c->gemm_items_stil.clear();
  c->gj_x.clear();
  c->gj_t.clear();
  c->itA.clear(); c->itC.clear(); c->itE.clear(); c->itF.clear(); c->itH.clear();
  c->itSA.clear(); c->itSC.clear(); c->itRA.clear();
  c->kig_ptr.clear(); c->kig_col.clear(); c->cgroups.clear(); c->cg_rows.clear(); c->cg_lds = 16;
  c->np_total = c->tp_total = 0;
  // packed symmetric blocks: forced (2), or (1) when they cut the operator bytes by a tenth or more
  // (blocks spanning several panels; a single panel holds the whole block anyway)
  c->packed = false;
  if (c->sym && c->opt.packed_sym != 0) {
    double full = 0.0, pk = 0.0;
    // the saving of storing the symmetric blocks once (several panels per block; with one panel the
    // tile kernels have too little parallelism for what the packing saves)
    for (const SubLayout& L : P.subs) {
      full += (double)round_up(L.nI + L.nG, 4) * L.nI + (double)round_up(L.nG + L.nc, 4) * L.nG;
      pk += (double)SymPack::elems(L.nI, L.nI + L.nG) + (double)SymPack::elems(L.nG, L.nG + L.nc);
    }
    c->packed = c->opt.packed_sym == 2 || pk <= 0.9 * full;
  }
  c->max_cols = 1;
  std::vector<GemmDesc> dS, dSs, dPhi, dStil;
  for (int64_t s = 0; s < P.n_sub; ++s) {
    const SubLayout& L = P.subs[s];
    SubDev& d = c->subs[s];
    d.nI = L.nI; d.nG = L.nG; d.nc = L.nc; d.inst = L.inst;
    d.n_elems = L.n_elems; d.ldK = L.ni();
    d.dof_off = L.dof_off; d.if_off = L.if_off; d.c_off = L.c_off; d.elem_off = L.elem_off; d.cons_off = L.cons_off;
    const int64_t ni = L.ni(), nI = L.nI, nG = L.nG, nc = L.nc, m = L.mP();
    // the symmetric path sweeps matrices beyond the one-workgroup kernels with the batched
    // blocked kernels (FP64 or FP32); the general path inverts blocks up to kGjMax rows in one
    // workgroup, larger ones (FP64 factorisations only) by the multi-workgroup pivoted Gauss-Jordan
    if (!c->sym && c->fact32 && std::max<int64_t>(nI, m) > kGjMax) return MBDDC_ERR_UNSUPPORTED;
    d.oK = w; w += round_up(ni * ni, 64);
    d.oG = w; w += round_up(nG * nI, 64);
    d.oH = w;
    if (!c->sym) w += round_up(nI * nG, 64);   // H = G^T on the symmetric path, never formed
    d.oP = w; w += round_up(m * m, 64);
    d.ld1 = (int32_t)round_up(nI + nG, 4);
    d.ld2 = (int32_t)round_up(nG + nc, 4);
    d.ld3 = (int32_t)round_up(nG, 4);
    d.ld4 = (int32_t)round_up(nI, 4);
    for (int q = 0; q < 2; ++q) d.oS[q] = d.oNP[q] = d.oTP[q] = -1;
    d.oNPA = -1;
    d.oKig = d.kig_ptr = d.kig_col = -1;
    if (c->sym) col_groups(P, L, (int32_t)s, c->cgroups, c->cg_rows);
    if (c->packed) {   // symmetric blocks stored once (SymPack), with their partial-product buffers
      d.ld1 = (int32_t)round_up(nG, 32);   // G alone (column-major, 128-byte aligned columns) for phase A
      d.oB1 = op; op += round_up((int64_t)d.ld1 * nI, 64);
      d.oNPA = c->np_total;
      c->np_total += (int64_t)nG * SymPack::panels((int32_t)nI);
      for (int32_t pp = 0; pp < SymPack::panels((int32_t)nI); ++pp)
        for (int32_t k = 0; k * kSymPanel < nG; ++k)
          c->itRA.push_back({(int32_t)s, k * kSymPanel, pp * kSymPanel,
                             std::min<int32_t>(kSymPanel, (int32_t)nG - k * kSymPanel)});
      d.oB2 = -1;
      const int32_t nS[2] = {(int32_t)nI, (int32_t)nG}, nr[2] = {(int32_t)nI, (int32_t)(nG + nc)};
      for (int q = 0; q < 2; ++q) {
        d.oS[q] = op;
        op += round_up(SymPack::elems(nS[q], nr[q]), 64);
        d.oNP[q] = c->np_total;
        c->np_total += SymPack::np_rows(nS[q], nr[q]);
        d.oTP[q] = c->tp_total;
        c->tp_total += SymPack::tp_count(SymPack::panels(nS[q])) * kSymPanel;
        const int32_t P = SymPack::panels(nS[q]), KT = (nr[q] + kSymPanel - 1) / kSymPanel;
        for (int32_t pp = 0; pp < P; ++pp)
          for (int32_t k = pp; k < KT; ++k)
            (q == 0 ? c->itSA : c->itSC).push_back({(int32_t)s, k * kSymPanel, pp * kSymPanel,
                                                   std::min<int32_t>(kSymPanel, nr[q] - k * kSymPanel)});
      }
    } else {
      d.oB1 = op; op += round_up((int64_t)d.ld1 * nI, 64);
      d.oB2 = op; op += round_up((int64_t)d.ld2 * nG, 64);
    }
    d.oB3 = op; op += round_up((int64_t)d.ld3 * nc, 64);
    if (c->packed) {
      d.oB4 = -1;
      const int64_t nnz = kig_pattern(P, L, c->kig_ptr, c->kig_col, d);
      d.oKig = op; op += round_up(nnz, 64);
    } else {
      d.oB4 = op; op += round_up((int64_t)d.ld4 * nG, 64);
    }
    d.oKc = kcl; kcl += nc * nc;
    d.oPiv = piv; piv += nI + m;
    c->max_cols = std::max<int>(c->max_cols, (int)std::max(std::max(nI, nG), nc));
    if (!c->sym && nI > kGjMax) c->gj_kii_large.push_back({d.oK, (int32_t)nI, (int32_t)ni, d.oPiv, (int32_t)s, 0});
    else c->gj_kii.push_back({d.oK, (int32_t)nI, (int32_t)ni, d.oPiv, (int32_t)s, 0});
    if (!c->sym && m > kGjMax) c->gj_p_large.push_back({d.oP, (int32_t)m, (int32_t)m, d.oPiv + nI, (int32_t)s, 0});
    else c->gj_p.push_back({d.oP, (int32_t)m, (int32_t)m, d.oPiv + nI, (int32_t)s, 0});
    // the blocked inverse stages kCoarseBlock rows at the matrix's row stride (ni for K_II)
    if (!c->sym) c->gen_large_max = std::max<int32_t>(c->gen_large_max, (int32_t)std::max<int64_t>(
                                       nI > kGjMax ? ni : 0, m > kGjMax ? m : 0));
    c->gj_x.push_back({d.oP, (int32_t)nG, (int32_t)nG, 0, (int32_t)s, 0});
    if (c->sym)   // T = C X C^T, inverted by the batched sweep
      c->gj_t.push_back({d.oP + nG * nG + 2 * nG * nc, (int32_t)nc, (int32_t)nc, 0, (int32_t)s, 0});
    // G = K_GI K_II^-1, H = K_II^-1 K_IG, S = K_GG - G K_IG
    GemmDesc g{};
    g.M = (int32_t)nG; g.N = (int32_t)nI; g.K = (int32_t)nI; g.lda = (int32_t)ni; g.ldb = (int32_t)ni; g.ldc = (int32_t)nI;
    g.ldci = 1; g.oA = d.oK + nI * ni; g.oB = d.oK; g.oC = d.oG; g.oCi = 0; g.alpha = 1.0; g.beta = 0.0;
    GemmDesc h{};
    h.M = (int32_t)nI; h.N = (int32_t)nG; h.K = (int32_t)nI; h.lda = (int32_t)ni; h.ldb = (int32_t)ni; h.ldc = (int32_t)nG;
    h.ldci = 1; h.oA = d.oK; h.oB = d.oK + nI; h.oC = d.oH; h.oCi = 0; h.alpha = 1.0; h.beta = 0.0;
    GemmDesc sS{};
    sS.M = (int32_t)nG; sS.N = (int32_t)nG; sS.K = (int32_t)nI; sS.lda = (int32_t)nI; sS.ldb = (int32_t)ni;
    sS.ldc = (int32_t)m; sS.ldci = (int32_t)ni; sS.oA = d.oG; sS.oB = d.oK + nI; sS.oC = d.oP;
    sS.oCi = d.oK + nI * ni + nI; sS.alpha = -1.0; sS.beta = 1.0;
    for (GemmDesc* gd : {&g, &h}) {
      int32_t tm = (int32_t)((gd->M + 63) / 64), tn = (int32_t)((gd->N + 63) / 64);
      gd->tiles_n = tn;
      int32_t id = (int32_t)c->gemm_desc.size();
      c->gemm_desc.push_back(*gd);
      for (int32_t a = 0; a < tm; ++a)
        for (int32_t b = 0; b < tn; ++b) {
          c->gemm_items_gh.push_back({id, a, b, 0});
          if (gd == &g) c->gemm_items_g.push_back({id, a, b, 0});
        }
    }
    sS.tiles_n = (int32_t)((sS.N + 63) / 64);
    dS.push_back(sS);
    GemmDesc sX = sS;               // symmetric path: S written into the X block (ld nG)
    sX.ldc = (int32_t)nG;
    dSs.push_back(sX);
    // symmetric path: Phi = XC T^-1 and S~ = X - Phi XC^T inside the P block
    GemmDesc ph{};
    ph.M = (int32_t)nG; ph.N = (int32_t)nc; ph.K = (int32_t)nc; ph.lda = (int32_t)nc; ph.ldb = (int32_t)nc;
    ph.ldc = (int32_t)nc; ph.ldci = 1; ph.oA = d.oP + nG * nG; ph.oB = d.oP + nG * nG + 2 * nG * nc;
    ph.oC = d.oP + nG * nG + nG * nc; ph.oCi = 0; ph.alpha = 1.0; ph.beta = 0.0;
    ph.tiles_n = (int32_t)((nc + 63) / 64);
    dPhi.push_back(ph);
    GemmDesc st{};
    st.M = (int32_t)nG; st.N = (int32_t)nG; st.K = (int32_t)nc; st.lda = (int32_t)nc; st.ldb = (int32_t)nc;
    st.ldc = (int32_t)nG; st.ldci = (int32_t)nG; st.oA = d.oP + nG * nG + nG * nc; st.oB = d.oP + nG * nG;
    st.oC = d.oP; st.oCi = d.oP; st.alpha = -1.0; st.beta = 1.0; st.transB = 1;
    st.tiles_n = (int32_t)((nG + 63) / 64);
    dStil.push_back(st);
  }
  build_apply_items(c);
  for (GemmDesc& sS : dS) {
    int32_t id = (int32_t)c->gemm_desc.size();
    c->gemm_desc.push_back(sS);
    int32_t tm = (sS.M + 63) / 64, tn = sS.tiles_n;
    for (int32_t a = 0; a < tm; ++a)
      for (int32_t b = 0; b < tn; ++b) c->gemm_items_s.push_back({id, a, b, 0});
  }
  auto add_items = [&](std::vector<GemmDesc>& ds, std::vector<GemmItem>& items) {
    for (GemmDesc& g : ds) {
      int32_t id = (int32_t)c->gemm_desc.size();
      c->gemm_desc.push_back(g);
      int32_t tm = (g.M + 63) / 64, tn = g.tiles_n;
      for (int32_t a = 0; a < tm; ++a)
        for (int32_t b = 0; b < tn; ++b) items.push_back({id, a, b, 0});
    }
  };
  add_items(dSs, c->gemm_items_ssym);
  add_items(dPhi, c->gemm_items_phi);
  add_items(dStil, c->gemm_items_stil);
  CHK(build_deluxe(c));
  if (c->sym && !(c->set_kii.build(c->gj_kii, c->fact32, c->tune) && c->set_x.build(c->gj_x, c->fact32, c->tune) &&
                  c->set_t.build(c->gj_t, c->fact32, c->tune) && c->set_dlx.build(c->gj_dlx, false, c->tune)))
    return MBDDC_ERR_UNSUPPORTED;
  c->big_pbuf = 0;
  c->big_count = 0;
  for (const SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
    c->big_pbuf = std::max(c->big_pbuf, S->pbuf_elems);
    c->big_count = std::max(c->big_count, (int64_t)S->big.size());
  }
  c->w_elems = w;
  c->op_elems = op;
  c->kcl_elems = kcl;
  c->piv_elems = piv;
  // coarse problems per instance
  c->inst_coarse_off.assign(P.n_inst, 0);
  c->inst_kc_off.assign(P.n_inst, 0);
  c->inst_nc.assign(P.n_inst, 0);
  c->inst_kc_ld.assign(P.n_inst, 0);
  c->inst_nchunk.assign(P.n_inst, 1);
  c->gj_coarse_small.clear();
  c->coarse_large.clear();
  int64_t kc = 0;
  c->coarse_max_nc = 0;
  c->nchunk_max = 1;
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const Instance& in = P.inst[ii];
    c->inst_coarse_off[ii] = in.coarse_off;
    c->inst_nc[ii] = in.n_coarse;
    int32_t ld = (int32_t)round_up(std::max(in.n_coarse, 1), 4);
    c->inst_kc_ld[ii] = ld;
    c->inst_kc_off[ii] = kc;
    kc += round_up((int64_t)ld * std::max(in.n_coarse, 1), 64);
    c->coarse_max_nc = std::max(c->coarse_max_nc, in.n_coarse);
    const bool three = c->opt.levels == 3;
    int32_t nch = three ? 1 : std::max(1, (in.n_coarse + kCoarseChunk - 1) / kCoarseChunk);
    c->inst_nchunk[ii] = nch;
    c->nchunk_max = std::max(c->nchunk_max, nch);
    if (in.n_coarse > 0 && !three) {
      if (in.n_coarse <= kGjMax)
        c->gj_coarse_small.push_back({c->inst_kc_off[ii], in.n_coarse, ld, in.coarse_off, ii, 0});
      else
        c->coarse_large.push_back(ii);
    }
  }
  // coarse product items: 64 RL rows of one column chunk each, with the longest row blocks that
  // still give every CU two workgroups (small coarse problems take short blocks)
  c->coarse_rl = 1;
  for (int rl : {4, 2}) {
    int64_t items = 0;
    for (int32_t ii = 0; ii < P.n_inst; ++ii) {
      const int32_t nc = P.inst[ii].n_coarse;
      if (nc > 0 && c->opt.levels != 3) items += (int64_t)nblk(nc, 64 * rl) * nblk(nc, kCoarseChunk);
    }
    if (items >= 512) {
      c->coarse_rl = rl;
      break;
    }
  }
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const int32_t nc = P.inst[ii].n_coarse;
    if (nc <= 0 || c->opt.levels == 3) continue;
    for (int32_t r0 = 0; r0 < nc; r0 += 64 * c->coarse_rl)
      for (int32_t c0 = 0; c0 < nc; c0 += kCoarseChunk)
        c->itE.push_back({ii, r0, c0, std::min(kCoarseChunk, nc - c0)});
  }
  c->kc_elems = kc;
  c->coarse_inst.assign(P.n_coarse, 0);
  for (int32_t ii = 0; ii < P.n_inst; ++ii)
    for (int32_t k = 0; k < P.inst[ii].n_coarse; ++k) c->coarse_inst[P.inst[ii].coarse_off + k] = ii;
  c->cslot_sub.assign(P.n_cslots, 0);
  for (int64_t s = 0; s < P.n_sub; ++s)
    for (int32_t k = 0; k < P.subs[s].nc; ++k) c->cslot_sub[P.subs[s].c_off + k] = (int32_t)s;
  // Krylov row chunks (never straddling an instance)
  c->chunk_inst.clear();
  c->chunk_begin.clear();
  c->inst_chunk_off.assign(P.n_inst + 1, 0);
  int64_t target = std::max<int64_t>(256, round_up(P.n_dofs / 1024 + 1, 64));
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    c->inst_chunk_off[ii] = (int32_t)c->chunk_inst.size();
    int64_t b0 = 3 * P.inst[ii].node_off, b1 = b0 + 3LL * P.inst[ii].n_nodes;
    for (int64_t b = b0; b < b1; b += target) {
      c->chunk_inst.push_back(ii);
      c->chunk_begin.push_back(b);
    }
  }
  c->inst_chunk_off[P.n_inst] = (int32_t)c->chunk_inst.size();
  c->chunk_begin.push_back(P.n_dofs);
  c->nblocks = (int64_t)P.bsr_col.size();
  for (const ColGroup& g : c->cgroups)
    c->cg_lds = std::max(c->cg_lds, (size_t)g.nu * (kCgW * sizeof(double) + sizeof(int32_t)));
  if (c->cg_lds > 159 * 1024) return MBDDC_ERR_UNSUPPORTED;   // an interface DOF coupled to > 1200 interior DOFs
  // algorithmic bytes (operators once) and flops of each launch family
  for (int f = 0; f < F_COUNT; ++f) c->op_bytes[f] = c->vec_words[f] = c->fam_flops[f] = 0.0;
  const double eo = (double)elem_size(c->mixed), ef = (double)elem_size(c->fact32);
  for (const SubDev& d : c->subs) {
    const double nI = d.nI, nG = d.nG, nc = d.nc, m = d.nG + d.nc;
    if (c->packed) {
      // A: G r_I; H: the slots' averages and r_I - K_IG z_G (prep), then K_II^-1 of it
      const double nnz = (double)(c->kig_ptr[d.kig_ptr + d.nI]);
      c->op_bytes[F_APPLY_A] += eo * d.ld1 * nI;
      c->op_bytes[F_APPLY_C] += eo * SymPack::elems(d.nG, d.nG + d.nc);
      c->op_bytes[F_APPLY_H] += eo * SymPack::elems(d.nI, d.nI);
      c->op_bytes[F_APPLY_HPREP] += (eo + 4.0) * nnz + 4.0 * (nI + 1);
      c->fam_flops[F_APPLY_A] += nG * nI;
      c->fam_flops[F_APPLY_H] += nI * nI;
      c->fam_flops[F_APPLY_HPREP] += nnz;
      c->vec_words[F_APPLY_A] += nI + nG;
      c->vec_words[F_APPLY_H] += 2 * nI;
      c->vec_words[F_APPLY_HPREP] += 3 * nG + 2 * nI;
    } else {
      c->op_bytes[F_APPLY_A] += eo * d.ld1 * nI;
      c->op_bytes[F_APPLY_C] += eo * d.ld2 * nG;
      c->op_bytes[F_APPLY_H] += eo * d.ld4 * nG;
      c->fam_flops[F_APPLY_A] += (nI + nG) * nI;
      c->fam_flops[F_APPLY_H] += nI * nG;
      c->vec_words[F_APPLY_A] += 2 * nI + nG;
      c->vec_words[F_APPLY_H] += nG + 2 * nI;
    }
    c->op_bytes[F_APPLY_F] += eo * d.ld3 * nc;
    c->fam_flops[F_APPLY_C] += (nG + nc) * nG;
    c->fam_flops[F_APPLY_F] += nG * nc;
    c->vec_words[F_APPLY_C] += 2 * nG + nG + nc;
    c->vec_words[F_APPLY_F] += nc + 2 * nG;
    // a symmetric sweep updates one triangle (n^3 flops per inverse), Gauss-Jordan the whole matrix (2 n^3)
    c->fam_flops[F_GJ_KII] += (c->sym ? 1.0 : 2.0) * nI * nI * nI;
    c->fam_flops[F_GJ_P] += c->sym ? (double)nG * nG * nG : 2.0 * m * m * m;
    if (!c->sym) {   // dense G, H and S (symmetric path: the sparse products, below)
      c->fam_flops[F_GEMM_GH] += 4.0 * nG * nI * nI;
      c->fam_flops[F_GEMM_S] += 2.0 * nG * nG * nI;
    }
    c->op_bytes[F_ASSEMBLE_LOCAL] += ef * (nI + nG) * (nI + nG);
  }
  for (const ColGroup& g : c->cgroups) {   // flops of the products as run (the group's full width)
    c->fam_flops[F_GEMM_GH] += 2.0 * g.nu * kCgW * c->subs[g.sub].nI;
    c->fam_flops[F_GEMM_S] += 2.0 * g.nu * kCgW * c->subs[g.sub].nG;
  }
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const double nc = c->inst_nc[ii];
    c->op_bytes[F_APPLY_E] += 8.0 * c->inst_kc_ld[ii] * nc;
    c->fam_flops[F_APPLY_E] += nc * nc;
    c->vec_words[F_APPLY_E] += nc * (1 + c->inst_nchunk[ii]);
    if (nc > 0 && nc <= kGjMax && c->opt.levels != 3) c->fam_flops[F_COARSE_GJ_SMALL] += 2.0 * nc * nc * nc;
  }
  c->op_bytes[F_ASSEMBLE_LOCAL] += 8.0 * P.ke_total;
  c->op_bytes[F_ASSEMBLE_BSR] = 8.0 * P.ke_total + 72.0 * c->nblocks;
  c->op_bytes[F_SPMV] = 76.0 * c->nblocks + 4.0 * (P.n_nodes + 1);
  return MBDDC_OK;
}

int upload_plan(mbddc_ctx* c) {
  const Plan& P = c->plan;
  CHK(upload(c, &c->d_subs, c->subs));
  CHK(upload(c, &c->d_sub_dofs, P.sub_dofs));
  CHK(upload(c, &c->d_sub_elems, P.sub_elems));
  CHK(upload(c, &c->d_elem_npe, P.elem_npe));
  CHK(upload(c, &c->d_elem_ldof, P.elem_ldof));
  CHK(upload(c, &c->d_ke_off, P.ke_off));
  CHK(upload(c, &c->d_elem_ldof_off, P.elem_ldof_off));
  CHK(upload(c, &c->d_cons_ptr, P.cons_ptr));
  CHK(upload(c, &c->d_cons_idx, P.cons_idx));
  CHK(upload(c, &c->d_cons_w, P.cons_w));
  CHK(upload(c, &c->d_slot_dof, P.slot_dof));
  CHK(upload(c, &c->d_slot_ifx, P.slot_ifx));
  CHK(upload(c, &c->d_slot_w, P.slot_w));
  CHK(upload(c, &c->d_slot_owner, P.slot_owner));
  CHK(upload(c, &c->d_ifx_ptr, P.ifx_ptr));
  CHK(upload(c, &c->d_ifx_slots, P.ifx_slots));
  CHK(upload(c, &c->d_cslot_coarse, P.cslot_coarse));
  CHK(upload(c, &c->d_cslot_sub, c->cslot_sub));
  CHK(upload(c, &c->d_coarse_ptr, P.coarse_ptr));
  CHK(upload(c, &c->d_coarse_slots, P.coarse_slots));
  CHK(upload(c, &c->d_coarse_inst, c->coarse_inst));
  CHK(upload(c, &c->d_inst_coarse_off, c->inst_coarse_off));
  CHK(upload(c, &c->d_inst_kc_off, c->inst_kc_off));
  CHK(upload(c, &c->d_inst_nc, c->inst_nc));
  CHK(upload(c, &c->d_inst_kc_ld, c->inst_kc_ld));
  CHK(upload(c, &c->d_inst_nchunk, c->inst_nchunk));
  std::vector<int32_t> rownode(c->nblocks);
  for (int64_t n = 0; n < P.n_nodes; ++n)
    for (int32_t b = P.bsr_rowptr[n]; b < P.bsr_rowptr[n + 1]; ++b) rownode[b] = (int32_t)n;
  CHK(upload(c, &c->d_bsr_rowptr, P.bsr_rowptr));
  CHK(upload(c, &c->d_bsr_col, P.bsr_col));
  CHK(upload(c, &c->d_bsr_rownode, rownode));
  CHK(upload(c, &c->d_bsr_cptr, P.bsr_cptr));
  CHK(upload(c, &c->d_bsr_contrib, P.bsr_contrib));
  CHK(upload(c, &c->d_bsr_kstride, P.bsr_kstride));
  CHK(upload(c, &c->d_free, P.free_dof));
  std::vector<int32_t> dof_inst(P.n_dofs);
  for (int64_t d = 0; d < P.n_dofs; ++d) dof_inst[d] = P.dof_inst[d];
  CHK(upload(c, &c->d_dof_inst, dof_inst));
  CHK(upload(c, &c->d_gj_kii, c->gj_kii));
  CHK(upload(c, &c->d_gj_p, c->gj_p));
  CHK(upload(c, &c->d_gj_cs, c->gj_coarse_small));
  CHK(upload(c, &c->d_gemm_desc, c->gemm_desc));
  CHK(upload(c, &c->d_gemm_gh, c->gemm_items_gh));
  CHK(upload(c, &c->d_gemm_s, c->gemm_items_s));
  CHK(upload(c, &c->d_gemm_g, c->gemm_items_g));
  CHK(upload(c, &c->d_gemm_ssym, c->gemm_items_ssym));
  CHK(upload(c, &c->d_gemm_phi, c->gemm_items_phi));
  CHK(upload(c, &c->d_gemm_stil, c->gemm_items_stil));
  CHK(upload(c, &c->d_gj_x, c->gj_x));
  CHK(upload(c, &c->d_gj_t, c->gj_t));
  for (SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
    CHK(upload(c, &S->d_all, S->all));
    CHK(upload(c, &S->d_big, S->big));
    CHK(upload(c, &S->d_items, S->items));
    CHK(upload(c, &S->d_gd, S->gd));
    CHK(upload(c, &S->d_gitems, S->gitems));
  }
  CHK(dalloc(c, &c->d_rho, std::max<int64_t>(P.n_sub, 1)));
  CHK(upload(c, &c->d_itA, c->itA));
  CHK(upload(c, &c->d_itC, c->itC));
  CHK(upload(c, &c->d_itE, c->itE));
  CHK(upload(c, &c->d_itF, c->itF));
  CHK(upload(c, &c->d_itH, c->itH));
  CHK(upload(c, &c->d_itSA, c->itSA));
  CHK(upload(c, &c->d_itSC, c->itSC));
  CHK(upload(c, &c->d_itRA, c->itRA));
  if (c->packed) {
    CHK(upload(c, &c->d_kig_ptr, c->kig_ptr));
    CHK(upload(c, &c->d_kig_col, c->kig_col));
  }
  CHK(upload(c, &c->d_cgroups, c->cgroups));
  CHK(upload(c, &c->d_cg_rows, c->cg_rows));
  if (c->deluxe) {
    CHK(upload(c, &c->d_dlx_blk, c->dlx_blk));
    CHK(upload(c, &c->d_dlx_glob, c->dlx_glob));
    CHK(upload(c, &c->d_dlx_idx, c->dlx_idx));
    CHK(upload(c, &c->d_dlx_gblk, c->dlx_gblk));
    CHK(upload(c, &c->d_dlx_ent_blk, c->dlx_ent_blk));
    CHK(upload(c, &c->d_dlx_ent_pos, c->dlx_ent_pos));
    CHK(upload(c, &c->d_dlx_tmp_off, c->dlx_tmp_off));
    CHK(upload(c, &c->d_gemm_dlx, c->gemm_items_dlx));
    CHK(upload(c, &c->d_ones, std::vector<double>(std::max<int64_t>(P.n_slots, 1), 1.0)));
    CHK(dalloc(c, &c->d_dlx_S, std::max<int64_t>(c->dlx_s_elems, 1)));
    CHK(dalloc(c, &c->d_dlx_D, std::max<int64_t>(c->dlx_s_elems, 1)));
    CHK(dalloc(c, &c->d_dlx_T, std::max<int64_t>(c->dlx_t_elems, 1)));
    CHK(dalloc(c, &c->d_dlx_tmp, std::max<int64_t>(c->dlx_tmp_elems, 1)));
  }
  CHK(upload(c, &c->d_chunk_inst, c->chunk_inst));
  CHK(upload(c, &c->d_chunk_begin, c->chunk_begin));
  CHK(upload(c, &c->d_inst_chunk_off, c->inst_chunk_off));
  // numeric buffers
  const size_t es = elem_size(c->mixed);
  CHK(dalloc(c, &c->d_Ke, P.ke_total));
  CHK(dalloc(c, &c->d_vals, c->nblocks * 9));
  CHK(dalloc(c, reinterpret_cast<unsigned char**>(&c->d_W), c->w_elems * (int64_t)elem_size(c->fact32)));
  CHK(dalloc(c, reinterpret_cast<unsigned char**>(&c->d_Op), c->op_elems * (int64_t)es));
  CHK(dalloc(c, &c->d_Kcl, c->kcl_elems));
  CHK(dalloc(c, &c->d_Kc, c->opt.levels == 3 ? 1 : c->kc_elems));
  if (c->opt.keep_coarse_matrix) CHK(dalloc(c, &c->d_Kc_keep, c->kc_elems));
  CHK(dalloc(c, &c->d_piv, c->piv_elems));
  c->status_len = std::max<int64_t>(std::max<int64_t>(P.n_sub, (int64_t)c->gj_coarse_small.size()),
                                    (int64_t)c->gj_dlx.size()) + 1;
  CHK(dalloc(c, &c->d_status, c->status_len));
  CHK(dalloc(c, &c->d_piv_c, std::max<int64_t>(std::max<int64_t>(P.n_coarse, std::max(c->coarse_max_nc,
                                                                                          c->gen_large_max)), 1)));
  if (c->gen_large_max > 0 && c->coarse_large.empty()) {   // pivoted Gauss-Jordan of large local blocks
    const int64_t ldmax = round_up(c->gen_large_max, 4), cb = std::max(kCoarseBlock, kSymCB);
    CHK(dalloc(c, &c->d_cDinv, 2 * cb * cb));
    CHK(dalloc(c, &c->d_cY, cb * ldmax));
    CHK(dalloc(c, &c->d_cCcol, ldmax * cb));
  }
  if (!c->coarse_large.empty()) {
    int64_t ldmax = round_up(std::max(c->coarse_max_nc, c->gen_large_max), 4);
    const int64_t cb = std::max(kCoarseBlock, kSymCB);
    CHK(dalloc(c, &c->d_cDinv, 2 * cb * cb));
    CHK(dalloc(c, &c->d_cY, cb * ldmax));
    CHK(dalloc(c, &c->d_cCcol, ldmax * cb));
    // panel products U = W Dinv of the symmetric sweep, n x kSymCB per instance
    std::vector<GemmDesc> gds;
    std::vector<GemmItem> items;
    c->csym_item_off.assign(1, 0);
    for (int32_t ii : c->coarse_large) {
      GemmDesc gd{};
      gd.M = c->inst_nc[ii]; gd.N = kSymCB; gd.K = kSymCB; gd.lda = kSymCB; gd.ldb = kSymCB; gd.ldc = kSymCB;
      gd.ldci = kSymCB; gd.tiles_n = kSymCB / 64; gd.alpha = 1.0; gd.beta = 0.0;
      const int32_t id = (int32_t)gds.size();
      gds.push_back(gd);
      for (int a = 0; a < (gd.M + 63) / 64; ++a)
        for (int b = 0; b < gd.tiles_n; ++b) items.push_back({id, a, b, 0});
      c->csym_item_off.push_back((int64_t)items.size());
    }
    CHK(upload(c, &c->d_csym_gd, gds));
    CHK(upload(c, &c->d_csym_items, items));
  }
  CHK(dalloc(c, &c->d_amax, 2));   // [0]: max |A| of a blocked inversion, [1]: rho of an augmentation
  if (c->big_count > 0) {
    CHK(dalloc(c, &c->d_bpanel, c->big_pbuf));
    CHK(dalloc(c, &c->d_bdinv, c->big_count * kSymCB * kSymCB));
    CHK(dalloc(c, &c->d_bthr, c->big_count));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

// Multilevel BDDC (§3.2, last paragraph): the coarse problem of every instance
// becomes a BDDC problem of its own. Level-2 nodes are the instance's fine
// primal globs (in glob order), each with the three components of a
// displacement; a component without a coarse DOF is clamped. Level-2 elements
// are the fine subdomains (nodes: their primal globs, ascending), fine
// subdomain i belongs to level-2 subdomain i / coarse_group, and a level-2
// node carries the boundary tags of its glob's first node.
int build_level2_host(mbddc_ctx* c, const std::vector<MeshIn>& fine) {
  const Plan& P = c->plan;
  const int32_t group = c->opt.coarse_group;
  std::vector<MeshIn> m2(P.n_inst);
  c->l2_dof.assign(P.n_coarse, -1);
  c->l2_eidx.assign(P.n_cslots, -1);
  int64_t node_off2 = 0;
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const Instance& in = P.inst[ii];
    if (in.n_coarse <= 0) return MBDDC_ERR_UNSUPPORTED;   // nothing to coarsen
    MeshIn& m = m2[ii];
    std::vector<int32_t> gnode(in.n_globs, -1);
    int32_t nn = 0;
    for (int32_t k = 0; k < in.n_coarse; ++k) {
      const int64_t cid = in.coarse_off + k;
      const int32_t g = P.coarse_glob[cid] - (int32_t)in.glob_off;
      if (gnode[g] < 0) gnode[g] = nn++;
      c->l2_dof[cid] = (int32_t)(3 * (node_off2 + gnode[g]) + P.coarse_comp[cid]);
    }
    m.n_nodes = nn;
    std::vector<uint8_t> present(3 * (size_t)nn, 0);
    for (int32_t k = 0; k < in.n_coarse; ++k) present[c->l2_dof[in.coarse_off + k] - 3 * node_off2] = 1;
    for (int32_t d = 0; d < 3 * nn; ++d)
      if (!present[d]) m.dirichlet.push_back(d);
    const std::vector<uint32_t>& tags = fine[ii].node_tags;
    if (!tags.empty()) {
      m.node_tags.assign(nn, 0u);
      for (int32_t g = 0; g < in.n_globs; ++g)
        if (gnode[g] >= 0) m.node_tags[gnode[g]] = tags[P.glob_node0[in.glob_off + g] - in.node_off];
    }
    m.n_elems = in.n_sub;
    m.n_sub = (in.n_sub + group - 1) / group;
    m.npe = 0;
    m.elem_ptr.push_back(0);
    for (int32_t i = 0; i < in.n_sub; ++i) {
      const SubLayout& L = P.subs[in.sub_off + i];
      if (L.nc <= 0) return MBDDC_ERR_UNSUPPORTED;        // a subdomain without primal DOFs
      std::vector<int32_t> nodes;
      for (int32_t p = 0; p < L.nc; ++p) {
        const int32_t cid = P.cslot_coarse[L.c_off + p];
        nodes.push_back((int32_t)(c->l2_dof[cid] / 3 - node_off2));
      }
      std::sort(nodes.begin(), nodes.end());
      nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
      for (int32_t p = 0; p < L.nc; ++p) {
        const int32_t cid = P.cslot_coarse[L.c_off + p];
        const int32_t nd = (int32_t)(c->l2_dof[cid] / 3 - node_off2);
        const int32_t a = (int32_t)(std::lower_bound(nodes.begin(), nodes.end(), nd) - nodes.begin());
        c->l2_eidx[L.c_off + p] = 3 * a + P.coarse_comp[cid];
      }
      m.elem_nodes.insert(m.elem_nodes.end(), nodes.begin(), nodes.end());
      m.elem_ptr.push_back((int32_t)m.elem_nodes.size());
      m.elem_part.push_back(i / group);
    }
    node_off2 += nn;
  }
  mbddc_ctx* ch = new (std::nothrow) mbddc_ctx();
  if (!ch) return MBDDC_ERR_OOM;
  c->child = ch;
  ch->device = c->device;
  ch->stream = c->stream;
  ch->alloc_fn = c->alloc_fn;
  ch->free_fn = c->free_fn;
  ch->alloc_user = c->alloc_user;
  ch->opt = c->opt;
  ch->opt.levels = 2;
  ch->opt.primal = c->opt.coarse_primal;
  ch->opt.precision = MBDDC_FP64;
  ch->opt.nnsp = 0;
  ch->opt.scaling = MBDDC_SCALING_COUNTING;
  ch->opt.packed_sym = 0;   // level-2 blocks: few panels, dense couplings; the full layout's fewer launches
  ch->mixed = false;
  ch->fact32 = false;
  ch->sym = c->sym;
  ch->tune = child_tuning(c->tune);
  if (!build_plan(m2, ch->opt.primal, ch->plan).empty()) return MBDDC_ERR_ARG;
  return build_layout(ch);
}

int upload_level2(mbddc_ctx* c) {
  mbddc_ctx* ch = c->child;
  CHK(upload_plan(ch));
  HIPCHK(hipMemsetAsync(ch->d_Ke, 0, ch->plan.ke_total * sizeof(double), c->stream));
  std::vector<int32_t> inv(std::max<int64_t>(ch->plan.n_dofs, 1), -1);
  for (int64_t k = 0; k < (int64_t)c->l2_dof.size(); ++k)
    if (c->l2_dof[k] >= 0) inv[c->l2_dof[k]] = (int32_t)k;
  CHK(upload(c, &c->d_l2_inv, inv));
  CHK(upload(c, &c->d_l2_eidx, c->l2_eidx));
  HIPCHK(hipStreamSynchronize(c->stream));
  ch->state = 2;
  return MBDDC_OK;
}

// Device bytes that a handle set up for `c`'s plan holds after factorisation and one
// solve with nrhs right-hand sides (host-side estimate for admission control).
double device_bytes_estimate(const mbddc_ctx* c, bool krylov, int nrhs) {
  const Plan& P = c->plan;
  const double es = (double)elem_size(c->mixed), ef = (double)elem_size(c->fact32);
  const double R = apply_R(nrhs), J = c->opt.restart + 1;
  double b = 8.0 * P.ke_total + 72.0 * c->nblocks + ef * c->w_elems + es * c->op_elems + 8.0 * c->kcl_elems;
  b += 8.0 * (c->opt.levels == 3 ? 0 : c->kc_elems) + (c->opt.keep_coarse_matrix ? 8.0 * c->kc_elems : 0.0);
  b += 4.0 * c->piv_elems;
  b += 4.0 * (P.sub_dofs.size() + P.sub_elems.size() + 2 * P.elem_npe.size() + P.elem_ldof.size());
  b += 8.0 * (P.ke_off.size() + P.elem_ldof_off.size() + P.cons_w.size() + P.slot_w.size() + P.bsr_contrib.size());
  b += 4.0 * (P.cons_idx.size() + P.cons_ptr.size() + 2 * P.slot_dof.size() + P.ifx_slots.size() + P.ifx_ptr.size());
  b += 4.0 * (2 * P.cslot_coarse.size() + P.coarse_slots.size() + P.coarse_ptr.size() + 2 * P.n_coarse);
  b += 4.0 * (P.bsr_rowptr.size() + 3 * P.bsr_col.size() + P.bsr_cptr.size()) + 5.0 * P.n_dofs;
  b += (double)sizeof(SubDev) * P.n_sub + 64.0 * (c->gj_kii.size() + c->gj_p.size() + c->gj_x.size());
  b += 48.0 * (c->gemm_desc.size()) + 16.0 * (c->gemm_items_gh.size() + c->gemm_items_s.size() +
       c->gemm_items_ssym.size() + c->gemm_items_phi.size() + c->gemm_items_stil.size());
  b += 16.0 * (c->itA.size() + c->itC.size() + c->itE.size() + c->itF.size() + c->itH.size() + c->itSA.size() +
               c->itSC.size() + c->itRA.size());
  b += 8.0 * R * (c->np_total + c->tp_total) + 4.0 * (c->kig_ptr.size() + c->kig_col.size()) +
       24.0 * c->cgroups.size() + 4.0 * c->cg_rows.size();
  if (c->deluxe)
    b += 8.0 * (2.0 * c->dlx_s_elems + c->dlx_t_elems + c->dlx_tmp_elems + c->dlx_tmp_off.size() + P.n_slots) +
         4.0 * (c->dlx_idx.size() + c->dlx_gblk.size() + 2.0 * P.n_slots) + 32.0 * c->dlx_blk.size() +
         24.0 * c->dlx_glob.size() + 48.0 * c->dlx_blk.size() + 16.0 * c->gemm_items_dlx.size();
  if (c->gen_large_max > 0 && c->coarse_large.empty()) {
    const double cb = std::max(kCoarseBlock, kSymCB), ld = round_up(c->gen_large_max, 4);
    b += 8.0 * (2 * cb * cb + 2 * cb * ld);
  }
  if (!c->coarse_large.empty()) {
    const double cb = std::max(kCoarseBlock, kSymCB), ld = round_up(std::max(c->coarse_max_nc, c->gen_large_max), 4);
    b += 8.0 * (2 * cb * cb + 2 * cb * ld);
  }
  if (c->big_count > 0) b += 8.0 * (c->big_pbuf + c->big_count * ((double)kSymCB * kSymCB + 1));
  for (const SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx})
    b += 32.0 * S->all.size() + 24.0 * S->big.size() + 8.0 * S->items.size() + 64.0 * S->gd.size() +
         16.0 * S->gitems.size();
  b += 8.0 * R * (2.0 * P.n_slots + std::max<int64_t>(P.n_cslots, 1) + c->nchunk_max * std::max<int64_t>(P.n_coarse, 1));
  b += 8.0 * R * P.n_dofs * (krylov ? (3 + 2 * J + 4) : 3);
  if (c->child) b += device_bytes_estimate(c->child, false, nrhs) + 8.0 * (P.n_coarse + P.n_cslots);
  return 1.02 * b + (1 << 20);
}

int ensure_apply_buffers(mbddc_ctx* c, int R) {
  if (c->child) CHK(ensure_apply_buffers(c->child, R));
  if (c->R_alloc >= R) {
    if (c->Y_R != R) {   // clamped entries of the output block are never written by the apply
      HIPCHK(hipMemsetAsync(c->d_Y, 0, c->plan.n_dofs * c->R_alloc * sizeof(double), c->stream));
      c->Y_R = R;
    }
    return MBDDC_OK;
  }
  const Plan& P = c->plan;
  dfree(c, c->d_tb); dfree(c, c->d_wb); dfree(c, c->d_cc); dfree(c, c->d_ep);
  dfree(c, c->d_X); dfree(c, c->d_Y); dfree(c, c->d_io);
  dfree(c, c->d_np); dfree(c, c->d_tp); dfree(c, c->d_cin);
  if (c->packed) {
    CHK(dalloc(c, &c->d_np, std::max<int64_t>(c->np_total, 1) * R));
    CHK(dalloc(c, &c->d_tp, std::max<int64_t>(c->tp_total, 1) * R));
    CHK(dalloc(c, &c->d_cin, std::max<int64_t>(P.n_ifx, 1) * R));
  }
  CHK(dalloc(c, &c->d_tb, P.n_slots * R));
  CHK(dalloc(c, &c->d_wb, P.n_slots * R));
  CHK(dalloc(c, &c->d_cc, std::max<int64_t>(P.n_cslots, 1) * R));
  CHK(dalloc(c, &c->d_ep, (int64_t)c->nchunk_max * std::max<int64_t>(P.n_coarse, 1) * R));
  CHK(dalloc(c, &c->d_X, P.n_dofs * R));
  CHK(dalloc(c, &c->d_Y, P.n_dofs * R));
  CHK(dalloc(c, &c->d_io, P.n_dofs * R));
  HIPCHK(hipMemsetAsync(c->d_Y, 0, P.n_dofs * R * sizeof(double), c->stream));
  c->R_alloc = R;
  c->Y_R = R;
  c->apply_gen++;
  return MBDDC_OK;
}

template <typename K>
int set_lds(K kern, size_t bytes) {
  static_assert(sizeof(K) > 0, "");
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return MBDDC_OK;
}

// ----------------------------------------------------------------------------
// numeric setup (factor)
// ----------------------------------------------------------------------------
// Batched GEMM: FP64 on the matrix cores when the tuning table says so, else on the vector units.
template <typename T>
void launch_gemm(mbddc_ctx* c, unsigned n_items, hipStream_t st, const GemmDesc* d, const GemmItem* it, const T* A,
                 const T* B, T* C, const T* Ci) {
  if (n_items == 0) return;
  if (c->tune.gemm_mfma) {
    hipLaunchKernelGGL((k_gemm_batched_mfma<T>), dim3(n_items), dim3(kBlock), 0, st, d, it, A, B, C, Ci);
    return;
  }
  hipLaunchKernelGGL((k_gemm_batched<T>), dim3(n_items), dim3(kBlock), 0, st, d, it, A, B, C, Ci);
}

template <typename T>
int run_gj(mbddc_ctx* c, T* base, const GjDesc* d_desc, int64_t count, int maxn, int32_t* d_stat, int32_t* d_pivs) {
  if (count == 0) return MBDDC_OK;
  constexpr int BP = sizeof(T) == 4 ? 32 : 16;
  size_t lds = ((size_t)maxn * (BP + 1) + (size_t)BP * maxn) * sizeof(T);
  lds = std::max<size_t>(lds, 16);
  CHK(set_lds(k_gj_batched<T, BP>, lds));
  hipLaunchKernelGGL((k_gj_batched<T, BP>), dim3((unsigned)count), dim3(kBlock), lds, c->stream, base, d_desc, d_pivs,
                     d_stat);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

template <typename T, int BP, bool MF>
int launch_sym(mbddc_ctx* c, T* base, const GjDesc* d_desc, int64_t count, int maxn, int32_t* d_stat) {
  const size_t lds = std::max<size_t>((size_t)2 * maxn * (BP + 1) * sizeof(T), 16);
  CHK(set_lds(k_sym_inv_batched<T, BP, MF>, lds));
  hipLaunchKernelGGL((k_sym_inv_batched<T, BP, MF>), dim3((unsigned)count), dim3(kBlock), lds, c->stream, base,
                     d_desc, d_stat);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

// Panels of 32 indices when both panel buffers fit in LDS (fewer passes over the
// matrix in memory), else of 16.
template <typename T>
int run_sym(mbddc_ctx* c, T* base, const GjDesc* d_desc, int64_t count, int maxn, int32_t* d_stat) {
  if (count == 0) return MBDDC_OK;
  if (sizeof(T) == 8 && maxn <= kSymRegMax) {   // the whole triangle fits in one workgroup's registers
    CHK(set_lds(k_sym_inv_reg, kSymRegLds));
    hipLaunchKernelGGL(k_sym_inv_reg, dim3((unsigned)count), dim3(kSymRegThreads), kSymRegLds, c->stream,
                       reinterpret_cast<double*>(base), d_desc, d_stat);
    HIPCHK(hipGetLastError());
    return MBDDC_OK;
  }
  if ((size_t)2 * maxn * 33 * sizeof(T) <= 159 * 1024) return launch_sym<T, 32, false>(c, base, d_desc, count, maxn, d_stat);
  return launch_sym<T, 16, false>(c, base, d_desc, count, maxn, d_stat);
}

// Inverts every matrix of a symmetric family in place (lower triangle read, full
// inverse written); statuses land in the set's slots.
template <typename T>
int run_symset(mbddc_ctx* c, T* base, const SymSet& S) {
  for (int v : {SV_REG, SV_BP16, SV_BP32}) {
    const int64_t cnt = S.grp_off[v + 1] - S.grp_off[v];
    if (cnt == 0) continue;
    const GjDesc* d = S.d_all + S.grp_off[v];
    int32_t* st = c->d_status + S.grp_off[v];
    if (v == SV_REG) {
      if (sizeof(T) != 8) return MBDDC_ERR_UNSUPPORTED;
      CHK(set_lds(k_sym_inv_reg, kSymRegLds));
      hipLaunchKernelGGL(k_sym_inv_reg, dim3((unsigned)cnt), dim3(kSymRegThreads), kSymRegLds, c->stream,
                         reinterpret_cast<double*>(base), d, st);
      HIPCHK(hipGetLastError());
    } else if (v == SV_BP16) {
      CHK((launch_sym<T, 16, false>(c, base, d, cnt, S.grp_maxn[v], st)));
    } else {
      CHK((launch_sym<T, 32, false>(c, base, d, cnt, S.grp_maxn[v], st)));
    }
  }
  if (S.big.empty()) return MBDDC_OK;
  // the panel and diagonal-inverse buffers are sized in doubles and hold T
  T* pbuf = reinterpret_cast<T*>(c->d_bpanel);
  T* dbuf = reinterpret_cast<T*>(c->d_bdinv);
  T* A = base;
  const unsigned nb = (unsigned)S.big.size();
  hipLaunchKernelGGL(k_bsym_prep<T>, dim3(nb), dim3(kBlock), 0, c->stream, S.d_big, A, c->d_bthr, c->d_status);
  CHK(set_lds(k_bsym_diag<T>, diag_lds<T>()));
  const int nmax = S.big[0].n;
  const unsigned gx = std::min<unsigned>(64, nblk((int64_t)nmax * kSymCB));
  unsigned active = nb;
  for (int k0 = 0; k0 < nmax; k0 += kSymCB) {
    while (active > 0 && S.big[active - 1].n <= k0) --active;
    hipLaunchKernelGGL(k_bsym_diag<T>, dim3(active), dim3(kBlock), diag_lds<T>(), c->stream, S.d_big, A, dbuf,
                       c->d_bthr, c->d_status, k0);
    hipLaunchKernelGGL(k_bsym_gather<T>, dim3(gx, active), dim3(kBlock), 0, c->stream, S.d_big, A, pbuf, k0);
    launch_gemm<T>(c, (unsigned)S.gitem_off[active], c->stream, S.d_gd, S.d_gitems, pbuf, dbuf, pbuf, pbuf);
    hipLaunchKernelGGL(k_bsym_update<T>, dim3((unsigned)S.item_off[active]), dim3(kBlock), 0, c->stream, S.d_big,
                       S.d_items, A, pbuf, dbuf, k0);
  }
  hipLaunchKernelGGL(k_bsym_finish<T>, dim3((unsigned)S.item_off[nb]), dim3(kBlock), 0, c->stream, S.d_big,
                     S.d_items, A);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

int check_status(mbddc_ctx* c, int64_t count, const std::vector<GjDesc>& descs, int* bad) {
  std::vector<int32_t> st(count);
  if (count == 0) return MBDDC_OK;
  HIPCHK(hipMemcpyAsync(st.data(), c->d_status, count * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < count; ++i)
    if (st[i] != 0) {
      *bad = descs[i].id;
      return MBDDC_ERR_SINGULAR;
    }
  return MBDDC_OK;
}

__global__ void k_absmax(const double* __restrict__ A, int n, int ld, double* out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n * n; i += (int64_t)gridDim.x * kBlock) {
    int r = (int)(i / n), cc = (int)(i % n);
    m = fmax(m, fabs(A[(int64_t)r * ld + cc]));
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(m));
}

// Symmetric coarse inverse: blocked sweep, lower triangle, MFMA update.
int coarse_sweep_large(mbddc_ctx* c, int32_t ii) {
  const int n = c->inst_nc[ii], ld = c->inst_kc_ld[ii];
  double* A = c->d_Kc + c->inst_kc_off[ii];
  HIPCHK(hipMemsetAsync(c->d_amax, 0, sizeof(double), c->stream));
  hipLaunchKernelGGL(k_absmax, dim3(512), dim3(kBlock), 0, c->stream, A, n, ld, c->d_amax);
  double amax = 0.0;
  HIPCHK(hipMemcpyAsync(&amax, c->d_amax, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemsetAsync(c->d_status, 0, sizeof(int32_t), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double thresh = std::max((double)n * 2.220446049250313e-16, 1e-12) * amax;
  double* Wg = c->d_cCcol;     // n x kSymCB
  double* Ug = c->d_cY;        // n x kSymCB
  const int64_t li = std::find(c->coarse_large.begin(), c->coarse_large.end(), ii) - c->coarse_large.begin();
  const GemmItem* d_items = c->d_csym_items + c->csym_item_off[li];
  const unsigned n_items = (unsigned)(c->csym_item_off[li + 1] - c->csym_item_off[li]);
  const unsigned nt = (unsigned)((n + 63) / 64);
  const unsigned ntiles = nt * (nt + 1) / 2;
  const unsigned nt2 = (unsigned)((n + kUpdTile - 1) / kUpdTile);
  const unsigned ntiles2 = nt2 * (nt2 + 1) / 2;
  const unsigned gg = std::min<unsigned>(2048, nblk((int64_t)n * kSymCB));
  if (!c->aux) {
    HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming));
  }
  const int nb = (n + kSymCB - 1) / kSymCB;
  double* Dbuf[2] = {c->d_cDinv, c->d_cDinv + kSymCB * kSymCB};
  // block 0: invert on the main stream
  CHK(set_lds(k_csym_diag, kDiagLds));
  hipLaunchKernelGGL(k_csym_diag, dim3(1), dim3(kBlock), kDiagLds, c->stream, A, n, ld, 0, Dbuf[0], c->d_status,
                     thresh);
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = kb * kSymCB;
    const int bw = std::min(kSymCB, n - k0);
    double* Dk = Dbuf[kb & 1];
    {
      ProfScope ps(c, F_COARSE_PREP, 16.0 * n * kSymCB, 2.0 * n * (double)kSymCB * kSymCB);
      hipLaunchKernelGGL(k_csym_gather, dim3(gg), dim3(kBlock), 0, c->stream, A, n, ld, k0, Wg);
      if (kb > 0) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_b, 0));     // Dinv of block kb (lookahead)
      launch_gemm<double>(c, (unsigned)(n_items), c->stream, c->d_csym_gd,
                         d_items, Wg, Dk, Ug, Ug);
    }
    const bool ahead = kb + 1 < nb;
    if (ahead) {
      // update diagonal block kb+1 first, then invert it on the lookahead stream
      hipLaunchKernelGGL(k_csym_update<1>, dim3(3), dim3(kBlock), 0, c->stream, A, n, ld, k0, Ug, Wg, Dk, kb + 1);
      HIPCHK(hipEventRecord(c->ev_a, c->stream));
      HIPCHK(hipStreamWaitEvent(c->aux, c->ev_a, 0));
      hipLaunchKernelGGL(k_csym_diag, dim3(1), dim3(kBlock), kDiagLds, c->aux, A, n, ld, k0 + kSymCB, Dbuf[(kb + 1) & 1],
                         c->d_status, thresh);
      HIPCHK(hipEventRecord(c->ev_b, c->aux));
    }
    {
      // algorithmic: lower-triangle read+write of A, flops 2 bw per lower entry
      const double lower = 0.5 * n * (double)(n + 1);
      ProfScope ps(c, F_COARSE_GEMM, 16.0 * lower, 2.0 * bw * lower);
      hipLaunchKernelGGL(k_csym_update<0>, dim3(ntiles2), dim3(kBlock), 0, c->stream, A, n, ld, k0, Ug, Wg, Dk,
                         ahead ? kb + 1 : -1);
    }
  }
  {
    ProfScope ps(c, F_COARSE_ROWS, 16.0 * n * (double)n, 0.0);
    hipLaunchKernelGGL(k_csym_finish, dim3(ntiles), dim3(kBlock), 0, c->stream, A, n, ld);
  }
  HIPCHK(hipGetLastError());
  int32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (st != 0) {
    c->last_bad = -1;
    return MBDDC_ERR_SINGULAR;
  }
  return MBDDC_OK;
}

// In-place inverse of one n x n FP64 matrix (row stride ld) by multi-workgroup Gauss-Jordan in
// blocks of kCoarseBlock pivots, each pivot the largest entry of its column within the diagonal
// block; *singular = 1 on a pivot below n eps max|A|. The rank-kCoarseBlock update descriptors
// are made once per matrix shape.
int invert_pivoted(mbddc_ctx* c, double* A, int n, int ld, int* singular);

int coarse_invert_large(mbddc_ctx* c, int32_t ii) {
  int sing = 0;
  CHK(invert_pivoted(c, c->d_Kc + c->inst_kc_off[ii], c->inst_nc[ii], c->inst_kc_ld[ii], &sing));
  if (sing) {
    c->last_bad = -1;
    return MBDDC_ERR_SINGULAR;
  }
  return MBDDC_OK;
}

int invert_pivoted(mbddc_ctx* c, double* A, int n, int ld, int* singular) {
  *singular = 0;
  HIPCHK(hipMemsetAsync(c->d_amax, 0, sizeof(double), c->stream));
  hipLaunchKernelGGL(k_absmax, dim3(512), dim3(kBlock), 0, c->stream, A, n, ld, c->d_amax);
  double amax = 0.0;
  HIPCHK(hipMemcpyAsync(&amax, c->d_amax, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemsetAsync(c->d_status, 0, sizeof(int32_t), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double thresh = (double)n * 2.220446049250313e-16 * amax;
  // single-problem GEMM descriptor re-used for every diagonal block (kept per shape)
  mbddc_ctx::PivGemm* pg = nullptr;
  for (auto& q : c->piv_gemm)
    if (q.n == n && q.ld == ld) pg = &q;
  if (!pg) {
    GemmDesc gd{};
    gd.M = n; gd.N = n; gd.K = kCoarseBlock; gd.lda = kCoarseBlock; gd.ldb = ld; gd.ldc = ld; gd.ldci = ld;
    gd.tiles_n = (n + 63) / 64; gd.oA = 0; gd.oB = 0; gd.oC = 0; gd.oCi = 0; gd.alpha = -1.0; gd.beta = 1.0;
    std::vector<GemmItem> its;
    for (int a = 0; a < (n + 63) / 64; ++a)
      for (int b = 0; b < gd.tiles_n; ++b) its.push_back({0, a, b, 0});
    mbddc_ctx::PivGemm q{n, ld, nullptr, nullptr, (int32_t)its.size()};
    CHK(upload(c, &q.d_gd, std::vector<GemmDesc>{gd}));
    CHK(upload(c, &q.d_items, its));
    c->piv_gemm.push_back(q);
    pg = &c->piv_gemm.back();
  }
  GemmDesc* d_gd = pg->d_gd;
  GemmItem* d_items = pg->d_items;
  const int32_t n_items = pg->n_items;
  const unsigned ncb = nblk(n, 64);
  const double gemm_flops = 2.0 * n * (double)n * kCoarseBlock;
  for (int k0 = 0; k0 < n; k0 += kCoarseBlock) {
    {
      ProfScope ps(c, F_COARSE_DIAG, 0.0, 2.0 * kCoarseBlock * kCoarseBlock * (double)kCoarseBlock);
      hipLaunchKernelGGL(k_cgj_diag, dim3(1), dim3(kBlock), 0, c->stream, A, n, ld, k0, c->d_cDinv, c->d_piv_c,
                         c->d_status, thresh);
    }
    {
      ProfScope ps(c, F_COARSE_PREP, 0.0, 2.0 * kCoarseBlock * kCoarseBlock * (double)n);
      hipLaunchKernelGGL(k_cgj_prep, dim3(ncb), dim3(kBlock), 0, c->stream, A, n, ld, k0, c->d_cDinv, c->d_piv_c,
                         c->d_cY, c->d_cCcol);
      hipLaunchKernelGGL(k_cgj_clear_panel, dim3(std::min<unsigned>(1024, nblk((int64_t)n * kCoarseBlock))),
                         dim3(kBlock), 0, c->stream, A, n, ld, k0);
    }
    {
      ProfScope ps(c, F_COARSE_GEMM, 16.0 * n * (double)n, gemm_flops);
      launch_gemm<double>(c, (unsigned)n_items, c->stream, d_gd, d_items, c->d_cCcol, c->d_cY, A, A);
    }
    {
      ProfScope ps(c, F_COARSE_ROWS, 0.0, 0.0);
      hipLaunchKernelGGL(k_cgj_rows, dim3(std::min<unsigned>(1024, nblk((int64_t)n * kCoarseBlock))), dim3(kBlock), 0,
                         c->stream, A, n, ld, k0, c->d_cY);
    }
  }
  hipLaunchKernelGGL(k_cgj_unswap, dim3(ncb, (unsigned)((n + kCoarseBlock - 1) / kCoarseBlock)), dim3(kBlock), 0,
                     c->stream, A, n, ld, c->d_piv_c);
  HIPCHK(hipGetLastError());
  int32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *singular = st != 0;
  return MBDDC_OK;
}

// General path: the local blocks above kGjMax rows, one matrix at a time. Constrained interface
// matrices (constrained = true) are augmented around the inversion (k_gen_augment).
template <typename T>
int run_gj_large(mbddc_ctx* c, T* W, const std::vector<GjDesc>& descs, int fam, bool constrained) {
  if (descs.empty()) return MBDDC_OK;
  if (!std::is_same<T, double>::value) return MBDDC_ERR_UNSUPPORTED;
  for (const GjDesc& d : descs) {
    int sing = 0;
    double* A = reinterpret_cast<double*>(W) + d.off;
    const int nc = constrained ? c->subs[d.id].nc : 0, nG = d.n - nc;
    {
      ProfScope ps(c, fam, 0.0, 2.0 * (double)d.n * d.n * d.n);
      if (nc > 0) {
        hipLaunchKernelGGL(k_gen_rho, dim3(1), dim3(kBlock), 0, c->stream, A, nG, d.ld, c->d_amax + 1);
        hipLaunchKernelGGL(k_gen_augment, dim3(std::min<unsigned>(2048, nblk((int64_t)nG * nG))), dim3(kBlock), 0,
                           c->stream, A, nG, nc, d.ld, c->d_amax + 1);
        HIPCHK(hipGetLastError());
      }
      CHK(invert_pivoted(c, A, d.n, d.ld, &sing));
      if (nc > 0 && !sing) {
        hipLaunchKernelGGL(k_gen_unaugment, dim3(nblk(nc)), dim3(kBlock), 0, c->stream, A, nG, nc, d.ld,
                           c->d_amax + 1);
        HIPCHK(hipGetLastError());
      }
    }
    if (sing) {
      c->last_bad = d.id;
      return MBDDC_ERR_SINGULAR;
    }
  }
  return MBDDC_OK;
}

// Deluxe weights from the Schur complements in the X blocks (before their augmentation): the glob
// blocks, their sums per glob, the sums' inverses and D = (sum S)^-1 S per block.
template <typename T>
int deluxe_weights(mbddc_ctx* c, T* W) {
  const unsigned nb = (unsigned)c->dlx_blk.size(), ng = (unsigned)c->dlx_glob.size();
  if (nb == 0) return MBDDC_OK;
  ProfScope ps(c, F_DELUXE, 0.0, 0.0);
  hipLaunchKernelGGL((k_dlx_gather<T>), dim3(nb), dim3(kBlock), 0, c->stream, c->d_subs, c->d_dlx_blk, c->d_dlx_idx,
                     W, c->d_dlx_S);
  hipLaunchKernelGGL(k_dlx_sum, dim3(ng), dim3(kBlock), 0, c->stream, c->d_dlx_glob, c->d_dlx_gblk, c->d_dlx_blk,
                     c->d_dlx_S, c->d_dlx_T);
  HIPCHK(hipGetLastError());
  CHK(run_symset<double>(c, c->d_dlx_T, c->set_dlx));
  int bad = 0;
  const int st = check_status(c, (int64_t)c->set_dlx.all.size(), c->set_dlx.all, &bad);
  if (st) {
    c->last_bad = -1;
    return st;
  }
  launch_gemm<double>(c, (unsigned)c->gemm_items_dlx.size(), c->stream, c->d_gemm_desc, c->d_gemm_dlx, c->d_dlx_T,
                      c->d_dlx_S, c->d_dlx_D, c->d_dlx_D);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

// S~ <- D S~ D^T and Phi <- D Phi per subdomain (through its scratch block).
template <typename T>
int deluxe_apply(mbddc_ctx* c, T* W) {
  if (c->dlx_blk.empty()) return MBDDC_OK;
  ProfScope ps(c, F_DELUXE, 0.0, 0.0);
  int64_t mx = 1;
  for (const SubDev& d : c->subs) mx = std::max<int64_t>(mx, (int64_t)d.nG * d.nG);
  const dim3 g((unsigned)std::min<int64_t>(64, (mx + 4 * kBlock - 1) / (4 * kBlock)), (unsigned)c->plan.n_sub);
  hipLaunchKernelGGL((k_dlx_right<T>), g, dim3(kBlock), 0, c->stream, c->d_subs, c->d_dlx_blk, c->d_dlx_idx,
                     c->d_dlx_ent_blk, c->d_dlx_ent_pos, c->d_dlx_D, W, c->d_dlx_tmp, c->d_dlx_tmp_off);
  hipLaunchKernelGGL((k_dlx_left<T>), g, dim3(kBlock), 0, c->stream, c->d_subs, c->d_dlx_blk, c->d_dlx_idx,
                     c->d_dlx_ent_blk, c->d_dlx_ent_pos, c->d_dlx_D, W, c->d_dlx_tmp, c->d_dlx_tmp_off);
  hipLaunchKernelGGL((k_dlx_phi<T, 0>), g, dim3(kBlock), 0, c->stream, c->d_subs, c->d_dlx_blk, c->d_dlx_idx,
                     c->d_dlx_ent_blk, c->d_dlx_ent_pos, c->d_dlx_D, W, c->d_dlx_tmp, c->d_dlx_tmp_off);
  hipLaunchKernelGGL((k_dlx_phi<T, 1>), g, dim3(kBlock), 0, c->stream, c->d_subs, c->d_dlx_blk, c->d_dlx_idx,
                     c->d_dlx_ent_blk, c->d_dlx_ent_pos, c->d_dlx_D, W, c->d_dlx_tmp, c->d_dlx_tmp_off);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

template <typename T, typename To>
int factor_impl(mbddc_ctx* c) {
  const Plan& P = c->plan;
  T* W = reinterpret_cast<T*>(c->d_W);
  To* Op = reinterpret_cast<To*>(c->d_Op);
  const unsigned nsub = (unsigned)P.n_sub;
  {
    ProfScope ps(c, F_ASSEMBLE_LOCAL, c->op_bytes[F_ASSEMBLE_LOCAL], 0.0);
    hipLaunchKernelGGL((k_assemble_local<T>), dim3(nsub), dim3(kBlock), 0, c->stream, c->d_Ke, c->d_subs,
                       c->d_sub_elems, c->d_ke_off, c->d_elem_npe, c->d_elem_ldof, c->d_elem_ldof_off, W);
  }
  HIPCHK(hipGetLastError());
  int maxI = 1, maxP = 1;   // the one-workgroup kernel's blocks (the general path's large ones go apart)
  for (const GjDesc& d : c->gj_kii) maxI = std::max(maxI, d.n);
  for (const GjDesc& d : c->gj_p) maxP = std::max(maxP, d.n);
  int bad = 0, st = 0;
  // K_II^-1 (interior / Dirichlet problems, §3.2 block factorisation)
  {
    ProfScope ps(c, F_GJ_KII, 0.0, c->fam_flops[F_GJ_KII]);
    if (c->sym) CHK(run_symset<T>(c, W, c->set_kii));
    else CHK(run_gj<T>(c, W, c->d_gj_kii, (int64_t)c->gj_kii.size(), maxI, c->d_status, c->d_piv));
  }
  st = c->sym ? check_status(c, (int64_t)c->set_kii.all.size(), c->set_kii.all, &bad)
              : check_status(c, (int64_t)c->gj_kii.size(), c->gj_kii, &bad);
  if (st) {
    c->last_bad = bad;
    return st;
  }
  if (!c->sym) CHK(run_gj_large<T>(c, W, c->gj_kii_large, F_GJ_KII, false));
  // G = K_GI K_II^-1 and H = K_II^-1 K_IG, S = K_GG - G K_IG: dense GEMMs on the general path;
  // on the symmetric path G^T = H and S = K_GG - K_GI G^T as sparse products over K_IG's pattern
  if (c->sym) {
    const unsigned ng = (unsigned)c->cgroups.size();
    if (ng > 0) {
      CHK(set_lds(k_kig_product<T, 0>, c->cg_lds));
      CHK(set_lds(k_kig_product<T, 1>, c->cg_lds));
      {
        ProfScope ps(c, F_GEMM_GH, 0.0, c->fam_flops[F_GEMM_GH]);
        hipLaunchKernelGGL((k_kig_product<T, 0>), dim3(ng), dim3(kBlock), c->cg_lds, c->stream, c->d_subs,
                           c->d_cgroups, c->d_cg_rows, W);
      }
      {
        ProfScope ps(c, F_GEMM_S, 0.0, c->fam_flops[F_GEMM_S]);
        hipLaunchKernelGGL((k_kig_product<T, 1>), dim3(ng), dim3(kBlock), c->cg_lds, c->stream, c->d_subs,
                           c->d_cgroups, c->d_cg_rows, W);
      }
    }
  } else {
    if (!c->gemm_items_gh.empty()) {
      ProfScope ps(c, F_GEMM_GH, 0.0, c->fam_flops[F_GEMM_GH]);
      launch_gemm<T>(c, (unsigned)c->gemm_items_gh.size(), c->stream, c->d_gemm_desc, c->d_gemm_gh, W, W, W, W);
    }
    if (!c->gemm_items_s.empty()) {
      ProfScope ps(c, F_GEMM_S, 0.0, c->fam_flops[F_GEMM_S]);
      launch_gemm<T>(c, (unsigned)c->gemm_items_s.size(), c->stream, c->d_gemm_desc, c->d_gemm_s, W, W, W, W);
    }
  }
  HIPCHK(hipGetLastError());
  if (c->sym) {
    if (c->deluxe) CHK(deluxe_weights<T>(c, W));
    // [S C^T; C 0]^-1 through X = (S + rho C^T C)^-1 and the constraint Schur complement
    {
      ProfScope ps(c, F_CONSTRAINTS, 0.0, 0.0);
      hipLaunchKernelGGL((k_add_ctc<T>), dim3(nsub), dim3(kBlock), 0, c->stream, c->d_subs, c->d_cons_ptr,
                         c->d_cons_idx, c->d_cons_w, W, c->d_rho);
    }
    {
      ProfScope ps(c, F_GJ_P, 0.0, c->fam_flops[F_GJ_P]);
      CHK(run_symset<T>(c, W, c->set_x));
    }
    st = check_status(c, (int64_t)c->set_x.all.size(), c->set_x.all, &bad);
    if (st) {
      c->last_bad = bad;
      return st;
    }
    {
      ProfScope ps(c, F_EXTRACT, 0.0, 0.0);
      {
        int64_t maxw = 1;   // largest n_G n_c of a subdomain: rows of stage 0 spread over workgroups
        for (const SubDev& d : c->subs) maxw = std::max<int64_t>(maxw, (int64_t)d.nG * d.nc);
        const unsigned parts = (unsigned)std::min<int64_t>(64, (maxw + 4 * kBlock - 1) / (4 * kBlock));
        hipLaunchKernelGGL((k_constraint_products<T, 0>), dim3(parts, nsub), dim3(kBlock), 0, c->stream, c->d_subs,
                           c->d_cons_ptr, c->d_cons_idx, c->d_cons_w, W);
        hipLaunchKernelGGL((k_constraint_products<T, 1>), dim3(1, nsub), dim3(kBlock), 0, c->stream, c->d_subs,
                           c->d_cons_ptr, c->d_cons_idx, c->d_cons_w, W);
      }
      HIPCHK(hipGetLastError());
      CHK(run_symset<T>(c, W, c->set_t));
      st = check_status(c, (int64_t)c->set_t.all.size(), c->set_t.all, &bad);
      if (st) {
        c->last_bad = bad;
        return st;
      }
      hipLaunchKernelGGL((k_tinv_finish<T>), dim3((unsigned)c->set_t.all.size()), dim3(kBlock), 0, c->stream,
                         c->d_subs, c->set_t.d_all, c->d_rho, W, c->d_Kcl);
      if (!c->gemm_items_phi.empty())
        launch_gemm<T>(c, (unsigned)c->gemm_items_phi.size(),
                           c->stream, c->d_gemm_desc, c->d_gemm_phi, W, W, W, W);
      if (!c->gemm_items_stil.empty())
        launch_gemm<T>(c, (unsigned)c->gemm_items_stil.size(),
                           c->stream, c->d_gemm_desc, c->d_gemm_stil, W, W, W, W);
      if (c->deluxe) CHK(deluxe_apply<T>(c, W));   // weights folded into S~ and Phi (extracted unweighted)
      const unsigned parts = (unsigned)std::min(64, std::max(1, (c->max_cols + 127) / 128));
      // the apply operators are not needed by the coarse problem: unless its families or the
      // extraction are being timed, they are written on a side stream while the coarse problem
      // (or the level-2 setup) is factorised on the handle's stream
      const uint32_t timed = (1u << F_EXTRACT) | (1u << F_LEVEL2_SETUP) | (1u << F_COARSE_ASSEMBLE) |
                             (1u << F_COARSE_GJ_SMALL) | (1u << F_COARSE_DIAG) | (1u << F_COARSE_PREP) |
                             (1u << F_COARSE_GEMM) | (1u << F_COARSE_ROWS);
      hipStream_t es = c->stream;
      if (P.n_coarse > 0 && !(c->prof.mask & timed)) {
        if (!c->side) {
          HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
          HIPCHK(hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(c->ev_side, c->stream));
        HIPCHK(hipStreamWaitEvent(c->side, c->ev_side, 0));
        es = c->side;
      }
      hipLaunchKernelGGL((k_extract_sym<T, To>), dim3(parts, nsub), dim3(kBlock), 0, es, c->d_subs,
                         c->deluxe ? c->d_ones : c->d_slot_w, c->d_kig_ptr, c->d_kig_col, W, Op);
      if (es != c->stream) {
        HIPCHK(hipEventRecord(c->ev_side, c->side));
        c->side_pending = true;
      }
    }
    HIPCHK(hipGetLastError());
  } else {
    {
      ProfScope ps(c, F_CONSTRAINTS, 0.0, 0.0);
      hipLaunchKernelGGL((k_build_constraints<T>), dim3(nsub), dim3(kBlock), 0, c->stream, c->d_subs, c->d_cons_ptr,
                         c->d_cons_idx, c->d_cons_w, W);
    }
    HIPCHK(hipGetLastError());
    {
      ProfScope ps(c, F_GJ_P, 0.0, c->fam_flops[F_GJ_P]);
      CHK(run_gj<T>(c, W, c->d_gj_p, (int64_t)c->gj_p.size(), maxP, c->d_status, c->d_piv));
    }
    st = check_status(c, (int64_t)c->gj_p.size(), c->gj_p, &bad);
    if (st) {
      c->last_bad = bad;
      return st;
    }
    CHK(run_gj_large<T>(c, W, c->gj_p_large, F_GJ_P, true));
    {
      ProfScope ps(c, F_EXTRACT, 0.0, 0.0);
      hipLaunchKernelGGL((k_extract<T, To>), dim3(nsub), dim3(kBlock), 0, c->stream, c->d_subs, c->d_slot_w, W, Op,
                         c->d_Kcl, c->opt.nonsym_coarse != 0 ? 1 : 0);
    }
  }
  // coarse problem (the extraction may still run on the side stream: joined below on every path)
  auto coarse_part = [&]() -> int {
  if (P.n_coarse > 0 && c->child) {
    // multilevel BDDC: S_PiPi is handed to the level-2 BDDC setup unassembled
    if (c->d_Kc_keep) {
      hipLaunchKernelGGL(k_coarse_assemble, dim3((unsigned)P.n_coarse), dim3(kBlock), 0, c->stream, c->d_subs,
                         c->d_coarse_ptr, c->d_coarse_slots, c->d_cslot_sub, c->d_cslot_coarse, c->d_inst_coarse_off,
                         c->d_inst_nc, c->d_inst_kc_off, c->d_inst_kc_ld, c->d_coarse_inst, c->d_Kcl, c->d_Kc_keep);
      HIPCHK(hipGetLastError());
    }
    mbddc_ctx* ch = c->child;
    {
      double f2 = 0.0;
      for (int f = 0; f < F_COUNT; ++f) f2 += ch->fam_flops[f];
      ProfScope ps(c, F_LEVEL2_SETUP, 0.0, f2);
      hipLaunchKernelGGL(k_l2_elements, dim3(nsub), dim3(kBlock), 0, c->stream, c->d_subs, c->d_Kcl, c->d_l2_eidx,
                         ch->d_ke_off, ch->d_elem_npe, ch->d_Ke);
      HIPCHK(hipGetLastError());
      ch->last_bad = 0;
      st = factor_impl<double, double>(ch);
    }
    if (st) {   // level-2 subdomain j -> -2 - j; level-3 coarse problem -> -2 - n_sub2
      c->last_bad = ch->last_bad >= 0 ? -2 - ch->last_bad : -2 - (int)ch->plan.n_sub;
      return st;
    }
    ch->state = 3;
  } else if (P.n_coarse > 0) {
    {
      ProfScope ps(c, F_COARSE_ASSEMBLE, 0.0, 0.0);
      hipLaunchKernelGGL(k_coarse_assemble, dim3((unsigned)P.n_coarse), dim3(kBlock), 0, c->stream, c->d_subs,
                         c->d_coarse_ptr, c->d_coarse_slots, c->d_cslot_sub, c->d_cslot_coarse, c->d_inst_coarse_off,
                         c->d_inst_nc, c->d_inst_kc_off, c->d_inst_kc_ld, c->d_coarse_inst, c->d_Kcl, c->d_Kc);
    }
    HIPCHK(hipGetLastError());
    if (c->d_Kc_keep)
      HIPCHK(hipMemcpyAsync(c->d_Kc_keep, c->d_Kc, c->kc_elems * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (!c->gj_coarse_small.empty()) {
      int maxc = 1;
      for (auto& g : c->gj_coarse_small) maxc = std::max(maxc, g.n);
      {
        ProfScope ps(c, F_COARSE_GJ_SMALL, 0.0, c->fam_flops[F_COARSE_GJ_SMALL]);
        if (c->sym)
          CHK(run_sym<double>(c, c->d_Kc, c->d_gj_cs, (int64_t)c->gj_coarse_small.size(), maxc, c->d_status));
        else
          CHK(run_gj<double>(c, c->d_Kc, c->d_gj_cs, (int64_t)c->gj_coarse_small.size(), maxc, c->d_status,
                             c->d_piv_c));
      }
      st = check_status(c, (int64_t)c->gj_coarse_small.size(), c->gj_coarse_small, &bad);
      if (st) {
        c->last_bad = -1;
        return st;
      }
    }
    for (int32_t ii : c->coarse_large) CHK(c->sym ? coarse_sweep_large(c, ii) : coarse_invert_large(c, ii));
  }
  return MBDDC_OK;
  };
  const int st_coarse = coarse_part();
  if (c->side_pending) {
    const hipError_t e = hipStreamWaitEvent(c->stream, c->ev_side, 0);
    c->side_pending = false;
    if (e != hipSuccess) return MBDDC_ERR_DEVICE;
  }
  if (st_coarse != MBDDC_OK) return st_coarse;
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

// ----------------------------------------------------------------------------
// preconditioner application and operator product on interleaved blocks
// ----------------------------------------------------------------------------
template <typename To, int R>
int apply_attrs();
// dynamic LDS of the packed tile kernel per right-hand side: cross-wave sums, the panel's and
// the row tile's inputs
constexpr size_t kSymLds = (4 * 256 + 2 * kSymPanel) * sizeof(double);
// of the rectangular tile kernel (phase A, packed path): cross-wave sums and the panel's inputs
constexpr size_t kRectLds = (4 * 256 + kSymPanel) * sizeof(double);

// Phase PH of the local apply (row-block list k of A, C, F, H) with that list's rows per
// workgroup: 256 (four rows per lane), 128 (two) or 64 (one).
template <typename To, int R, int PH>
void launch_local(mbddc_ctx* c, ApplyArgs a, int k, size_t n_items) {
  const int rw = c->apply_rows_eff[k];
  auto lds_of = [&](int x) { return (size_t)(4 * rw * R + (size_t)x * R) * sizeof(double); };
  // every input column in one LDS chunk when that keeps as many workgroups per CU as the tuned
  // chunk (fewer gather rounds and barriers; the narrow row blocks leave the LDS room)
  constexpr size_t kCuLds = 160 * 1024;
  if (c->max_cols > a.xchunk && kCuLds / lds_of(c->max_cols) >= kCuLds / lds_of(a.xchunk)) a.xchunk = c->max_cols;
  const size_t lds = lds_of(a.xchunk);
  const bool big = c->tune.apply_big > 0 || (c->tune.apply_big < 0 && c->max_cols >= kApplyBigCols);
  const dim3 g((unsigned)n_items), b(kBlock);
  if (rw == 64) hipLaunchKernelGGL((k_apply_local<To, R, PH, 1, false>), g, b, lds, c->stream, a);
  else if (rw == 128 && big) hipLaunchKernelGGL((k_apply_local<To, R, PH, 2, true>), g, b, lds, c->stream, a);
  else if (rw == 128) hipLaunchKernelGGL((k_apply_local<To, R, PH, 2, false>), g, b, lds, c->stream, a);
  else if (big) hipLaunchKernelGGL((k_apply_local<To, R, PH, 4, true>), g, b, lds, c->stream, a);
  else hipLaunchKernelGGL((k_apply_local<To, R, PH, 4, false>), g, b, lds, c->stream, a);
}

// z = M^-1 r. For the level-2 instance of a three-level handle (parent != null) the input
// is gathered from the parent's coarse slots and the output also written to the parent's
// coarse partial products, inside the level-2 phases.
template <typename To, int R>
int apply_impl(mbddc_ctx* c, const double* r, double* z, mbddc_ctx* parent = nullptr) {
  const Plan& P = c->plan;
  ApplyArgs a{};
  if (parent) {
    a.l2_inv = parent->d_l2_inv; a.l2_ptr = parent->d_coarse_ptr; a.l2_slots = parent->d_coarse_slots;
    a.l2_cc = parent->d_cc; a.l2_ep = parent->d_ep;
  }
  a.subs = c->d_subs; a.sub_dofs = c->d_sub_dofs; a.slot_dof = c->d_slot_dof; a.slot_ifx = c->d_slot_ifx;
  a.slot_owner = c->d_slot_owner; a.ifx_ptr = c->d_ifx_ptr; a.ifx_slots = c->d_ifx_slots;
  a.cslot_coarse = c->d_cslot_coarse; a.coarse_ptr = c->d_coarse_ptr; a.coarse_slots = c->d_coarse_slots;
  a.inst_nchunk = c->d_inst_nchunk; a.op = c->d_Op; a.kcinv = c->d_Kc; a.inst_kc_off = c->d_inst_kc_off;
  a.inst_kc_ld = c->d_inst_kc_ld; a.inst_coarse_off = c->d_inst_coarse_off; a.inst_nc = c->d_inst_nc;
  a.r = r; a.z = z; a.tb = c->d_tb; a.wb = c->d_wb; a.cc = c->d_cc; a.ep = c->d_ep; a.n_coarse = P.n_coarse;
  a.xchunk = std::min(c->max_cols, c->tune.xchunk);
  CHK((apply_attrs<To, R>()));
  if ((4 * 256 * R + (size_t)a.xchunk * R) * sizeof(double) > 160 * 1024) return MBDDC_ERR_UNSUPPORTED;
  a.np = c->d_np;
  a.tp = c->d_tp;
  a.cin = c->d_cin;
  a.n_ifx = P.n_ifx;
  a.kig_ptr = c->d_kig_ptr;
  a.kig_col = c->d_kig_col;
  a.n_slots = P.n_slots;
  {
    ProfScope ps(c, F_APPLY_A, c->op_bytes[F_APPLY_A] + 8.0 * R * c->vec_words[F_APPLY_A], 2.0 * R * c->fam_flops[F_APPLY_A]);
    if (c->packed) {   // G r_I alone: 256 x 256 tiles, then their panel sums
      a.items = c->d_itRA;
      if (!c->itRA.empty())
        hipLaunchKernelGGL((k_apply_rect<To, R>), dim3((unsigned)c->itRA.size()), dim3(kBlock), kRectLds * R,
                           c->stream, a);
    } else {
      a.items = c->d_itA;
      launch_local<To, R, 0>(c, a, 0, c->itA.size());
    }
  }
  if (c->packed) {
    ProfScope ps(c, F_APPLY_SYMRED, 0.0, 0.0);
    a.items = c->d_itA;
    hipLaunchKernelGGL((k_apply_rect_reduce<R>), dim3((unsigned)c->itA.size()), dim3(kBlock), 0, c->stream, a);
    if (P.n_ifx > 0) hipLaunchKernelGGL((k_c_prep<R>), dim3(nblk(P.n_ifx)), dim3(kBlock), 0, c->stream, a);
  }
  {
    ProfScope ps(c, F_APPLY_C, c->op_bytes[F_APPLY_C] + 8.0 * R * c->vec_words[F_APPLY_C], 2.0 * R * c->fam_flops[F_APPLY_C]);
    if (c->packed) {
      a.items = c->d_itSC;
      if (!c->itSC.empty())
        hipLaunchKernelGGL((k_apply_sym<To, R, 1>), dim3((unsigned)c->itSC.size()), dim3(kBlock), kSymLds * R, c->stream, a);
    } else {
      a.items = c->d_itC;
      launch_local<To, R, 1>(c, a, 1, c->itC.size());
    }
  }
  if (c->packed) {
    ProfScope ps(c, F_APPLY_SYMRED, 0.0, 0.0);
    a.items = c->d_itC;
    hipLaunchKernelGGL((k_apply_sym_reduce<R, 1>), dim3((unsigned)c->itC.size()), dim3(kBlock), 0, c->stream, a);
  }
  if (c->child) {
    mbddc_ctx* ch = c->child;
    double b2 = 16.0 * R * P.n_coarse, f2 = 0.0;   // coarse gather + scatter, then the level-2 phases
    for (int f : {F_APPLY_A, F_APPLY_C, F_APPLY_E, F_APPLY_F, F_APPLY_H, F_APPLY_HPREP}) {
      b2 += ch->op_bytes[f] + 8.0 * R * ch->vec_words[f];
      f2 += 2.0 * R * ch->fam_flops[f];
    }
    ProfScope ps(c, F_LEVEL2_APPLY, b2, f2);
    CHK((apply_impl<double, R>(ch, ch->d_X, ch->d_Y, c)));
  } else if (!c->itE.empty()) {
    const int rl = c->coarse_rl;
    const size_t lds_c = (size_t)(4 * 64 * rl * R + kCoarseChunk * R) * sizeof(double);
    ProfScope ps(c, F_APPLY_E, c->op_bytes[F_APPLY_E] + 8.0 * R * c->vec_words[F_APPLY_E],
                 2.0 * R * c->fam_flops[F_APPLY_E]);
    a.items = c->d_itE;
    const dim3 g((unsigned)c->itE.size()), b(kBlock);
    if (rl == 4) hipLaunchKernelGGL((k_apply_coarse<To, R, 4>), g, b, lds_c, c->stream, a);
    else if (rl == 2) hipLaunchKernelGGL((k_apply_coarse<To, R, 2>), g, b, lds_c, c->stream, a);
    else hipLaunchKernelGGL((k_apply_coarse<To, R, 1>), g, b, lds_c, c->stream, a);
  }
  {
    ProfScope ps(c, F_APPLY_F, c->op_bytes[F_APPLY_F] + 8.0 * R * c->vec_words[F_APPLY_F], 2.0 * R * c->fam_flops[F_APPLY_F]);
    a.items = c->d_itF;
    launch_local<To, R, 3>(c, a, 2, c->itF.size());
  }
  if (c->packed) {   // z_G, then z_I = K_II^-1 (r_I - K_IG z_G)
    {
      ProfScope ps(c, F_APPLY_HPREP, c->op_bytes[F_APPLY_HPREP] + 8.0 * R * c->vec_words[F_APPLY_HPREP],
                   2.0 * R * c->fam_flops[F_APPLY_HPREP]);
      if (P.n_slots > 0)
        hipLaunchKernelGGL((k_h_gather<R>), dim3(nblk(P.n_slots)), dim3(kBlock), 0, c->stream, a);
      a.items = c->d_itH;
      hipLaunchKernelGGL((k_h_prep<To, R>), dim3((unsigned)c->itH.size()), dim3(kBlock), 0, c->stream, a);
    }
    {
      ProfScope ps(c, F_APPLY_H, c->op_bytes[F_APPLY_H] + 8.0 * R * c->vec_words[F_APPLY_H],
                   2.0 * R * c->fam_flops[F_APPLY_H]);
      a.items = c->d_itSA;
      if (!c->itSA.empty())
        hipLaunchKernelGGL((k_apply_sym<To, R, 2>), dim3((unsigned)c->itSA.size()), dim3(kBlock), kSymLds * R, c->stream, a);
    }
    ProfScope ps(c, F_APPLY_SYMRED, 0.0, 0.0);
    a.items = c->d_itH;
    hipLaunchKernelGGL((k_apply_sym_reduce<R, 2>), dim3((unsigned)c->itH.size()), dim3(kBlock), 0, c->stream, a);
  } else {
    ProfScope ps(c, F_APPLY_H, c->op_bytes[F_APPLY_H] + 8.0 * R * c->vec_words[F_APPLY_H], 2.0 * R * c->fam_flops[F_APPLY_H]);
    a.items = c->d_itH;
    launch_local<To, R, 4>(c, a, 3, c->itH.size());
  }
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

int apply_dispatch(mbddc_ctx* c, int R, const double* r, double* z) {
  if (c->mixed) {
    switch (R) {
      case 1: return apply_impl<float, 1>(c, r, z);
      case 2: return apply_impl<float, 2>(c, r, z);
      case 4: return apply_impl<float, 4>(c, r, z);
      default: return apply_impl<float, 8>(c, r, z);
    }
  }
  switch (R) {
    case 1: return apply_impl<double, 1>(c, r, z);
    case 2: return apply_impl<double, 2>(c, r, z);
    case 4: return apply_impl<double, 4>(c, r, z);
    default: return apply_impl<double, 8>(c, r, z);
  }
}

// LDS attributes of the apply kernels for width R (set once per instantiation; outside
// any stream capture)
template <typename To, int R>
int apply_attrs() {
  static std::once_flag once;
  static int st = MBDDC_OK;
  std::call_once(once, [] {
    const size_t mx = 160 * 1024;
    int e = set_lds(k_apply_coarse<To, R, 4>, mx);
    if (!e) e = set_lds(k_apply_coarse<To, R, 2>, mx);
    if (!e) e = set_lds(k_apply_coarse<To, R, 1>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 0, 4, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 1, 4, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 3, 4, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 4, 4, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 0, 2, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 1, 2, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 3, 2, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 4, 2, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 0, 4, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 1, 4, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 3, 4, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 4, 4, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 0, 2, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 1, 2, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 3, 2, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 4, 2, true>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 0, 1, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 1, 1, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 3, 1, false>, mx);
    if (!e) e = set_lds(k_apply_local<To, R, 4, 1, false>, mx);
    if (!e) e = set_lds(k_apply_sym<To, R, 1>, mx);
    if (!e) e = set_lds(k_apply_sym<To, R, 2>, mx);
    if (!e) e = set_lds(k_apply_rect<To, R>, mx);
    st = e;
  });
  return st;
}

int apply_attrs_all(int R) {
  switch (R) {
    case 1: CHK((apply_attrs<float, 1>())); return apply_attrs<double, 1>();
    case 2: CHK((apply_attrs<float, 2>())); return apply_attrs<double, 2>();
    case 4: CHK((apply_attrs<float, 4>())); return apply_attrs<double, 4>();
    default: CHK((apply_attrs<float, 8>())); return apply_attrs<double, 8>();
  }
}

constexpr uint32_t kApplyFamilies = (1u << F_APPLY_A) | (1u << F_APPLY_C) | (1u << F_APPLY_E) | (1u << F_APPLY_F) |
                                    (1u << F_APPLY_H) | (1u << F_LEVEL2_APPLY) | (1u << F_APPLY_SYMRED) |
                                    (1u << F_APPLY_HPREP);

// z = M^-1 r on the handle's fixed blocks d_X -> d_Y: replayed from a captured graph
// unless graphs are off or an apply family is being profiled.
// Algorithmic bytes and flops of one whole preconditioner application with R right-hand sides
// (every phase, and the level-2 application when there is one).
void apply_totals(const mbddc_ctx* c, int R, double* bytes, double* flops) {
  double b = 0.0, f = 0.0;
  for (int k : {F_APPLY_A, F_APPLY_C, F_APPLY_F, F_APPLY_H, F_APPLY_HPREP}) {
    b += c->op_bytes[k] + 8.0 * R * c->vec_words[k];
    f += 2.0 * R * c->fam_flops[k];
  }
  if (const mbddc_ctx* ch = c->child) {
    b += 16.0 * R * c->plan.n_coarse;
    for (int k : {F_APPLY_A, F_APPLY_C, F_APPLY_E, F_APPLY_F, F_APPLY_H, F_APPLY_HPREP}) {
      b += ch->op_bytes[k] + 8.0 * R * ch->vec_words[k];
      f += 2.0 * R * ch->fam_flops[k];
    }
  } else if (!c->itE.empty()) {
    b += c->op_bytes[F_APPLY_E] + 8.0 * R * c->vec_words[F_APPLY_E];
    f += 2.0 * R * c->fam_flops[F_APPLY_E];
  }
  *bytes = b;
  *flops = f;
}

int apply_run(mbddc_ctx* c, int R) {
  c->n_applies++;
  double ab = 0.0, af = 0.0;
  if (c->prof.mask & (1u << F_APPLY_WHOLE)) apply_totals(c, R, &ab, &af);
  // brackets the whole application, eager or replayed from the graph (does not force eager launches)
  ProfScope whole(c, F_APPLY_WHOLE, ab, af);
  const bool profiled = (c->prof.mask & kApplyFamilies) || (c->child && (c->child->prof.mask & kApplyFamilies));
  if (!c->opt.graph_apply || profiled) return apply_dispatch(c, R, c->d_X, c->d_Y);
  const int slot = R == 1 ? 0 : (R == 2 ? 1 : (R == 4 ? 2 : 3));
  const int64_t gen = c->apply_gen + (c->child ? c->child->apply_gen : 0);
  hipGraphExec_t& ex = c->apply_exec[slot];
  if (ex && c->apply_exec_gen[slot] != gen) {
    HIPCHK(hipGraphExecDestroy(ex));
    ex = nullptr;
  }
  if (!ex) {
    CHK(apply_attrs_all(R));
    // captured on a private stream (the handle's stream may be the legacy default stream,
    // which cannot be captured); the graph is then launched on the handle's stream
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    if (c->child) c->child->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    int st = MBDDC_OK;
    if (e == hipSuccess) {
      st = apply_dispatch(c, R, c->d_X, c->d_Y);
      e = hipStreamEndCapture(c->cap_stream, &g);
    }
    c->stream = user;
    if (c->child) c->child->stream = user;
    if (st != MBDDC_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != MBDDC_OK ? st : MBDDC_ERR_DEVICE;
    }
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      ex = nullptr;
      return MBDDC_ERR_DEVICE;
    }
    c->apply_exec_gen[slot] = gen;
  }
  HIPCHK(hipGraphLaunch(ex, c->stream));
  c->n_applies_graphed++;
  return MBDDC_OK;
}

template <int G>
void launch_spmv(mbddc_ctx* c, int R, const double* x, double* y) {
  const int64_t nn = c->plan.n_nodes;
  const unsigned g = nblk(nn * G);
  switch (R) {
    case 1: hipLaunchKernelGGL((k_spmv<1, G>), dim3(g), dim3(kBlock), 0, c->stream, c->d_bsr_rowptr, c->d_bsr_col, c->d_vals, nn, x, y); break;
    case 2: hipLaunchKernelGGL((k_spmv<2, G>), dim3(g), dim3(kBlock), 0, c->stream, c->d_bsr_rowptr, c->d_bsr_col, c->d_vals, nn, x, y); break;
    case 4: hipLaunchKernelGGL((k_spmv<4, G>), dim3(g), dim3(kBlock), 0, c->stream, c->d_bsr_rowptr, c->d_bsr_col, c->d_vals, nn, x, y); break;
    default: hipLaunchKernelGGL((k_spmv<8, G>), dim3(g), dim3(kBlock), 0, c->stream, c->d_bsr_rowptr, c->d_bsr_col, c->d_vals, nn, x, y); break;
  }
}

int spmv_dispatch(mbddc_ctx* c, int R, const double* x, double* y) {
  const int64_t nd = c->plan.n_dofs, nn = c->plan.n_nodes;
  // 16-byte loads of x need a 16-byte aligned base (every block here comes from the allocator)
  if ((reinterpret_cast<uintptr_t>(x) & 15) != 0) return MBDDC_ERR_UNSUPPORTED;
  ProfScope ps(c, F_SPMV, c->op_bytes[F_SPMV] + 16.0 * R * nd, 18.0 * R * c->nblocks);
  // 32 lanes (10 blocks per pass) suit rows of about 27 blocks (trilinear elements); rows of about
  // 64 blocks and more (triquadratic elements) take a whole wave (21 blocks per pass)
  if (c->nblocks > kSpmvWideRow * nn)
    launch_spmv<64>(c, R, x, y);
  else
    launch_spmv<32>(c, R, x, y);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

// copies the API layout [nrhs][n] (host or device) into the interleaved block dst
int load_block(mbddc_ctx* c, const double* src, int nrhs, int R, int on_device, double* dst) {
  const int64_t n = c->plan.n_dofs;
  const double* s = src;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(c->d_io, src, (size_t)n * nrhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
    s = c->d_io;
  }
  hipLaunchKernelGGL(k_to_interleaved, dim3(nblk(n * R)), dim3(kBlock), 0, c->stream, s, nrhs, R, n, c->d_free, dst);
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

int store_block(mbddc_ctx* c, const double* src, int nrhs, int R, int on_device, double* dst) {
  const int64_t n = c->plan.n_dofs;
  double* d = on_device ? dst : c->d_io;
  hipLaunchKernelGGL(k_from_interleaved, dim3(nblk(n * nrhs)), dim3(kBlock), 0, c->stream, src, nrhs, R, n, d);
  HIPCHK(hipGetLastError());
  if (!on_device)
    HIPCHK(hipMemcpyAsync(dst, c->d_io, (size_t)n * nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

// ----------------------------------------------------------------------------
// GMRES
// ----------------------------------------------------------------------------
int ensure_krylov(mbddc_ctx* c, int R) {
  const int restart = c->opt.restart;
  if (c->R_kry >= R && c->restart_kry == restart) return MBDDC_OK;
  for (double** p : {&c->d_V, &c->d_Z, &c->d_Wv, &c->d_B, &c->d_x, &c->d_r, &c->d_part, &c->d_part2, &c->d_npart,
                     &c->d_h1, &c->d_h2, &c->d_Hs, &c->d_cs, &c->d_sn, &c->d_g, &c->d_hnorm, &c->d_y, &c->d_beta})
    dfree(c, *p);
  dfree(c, c->d_kstate); dfree(c, c->d_nk); dfree(c, c->d_fin); dfree(c, c->d_bnorm);
  c->d_jsys = c->d_its = nullptr;
  c->d_active = c->d_mode = nullptr;
  const int64_t n = c->plan.n_dofs, J = restart + 1;
  const int64_t nsys = (int64_t)c->plan.n_inst * R;
  if (nsys > c->h_cap) {   // pinned host buffers are kept while large enough (a host free syncs the device)
    if (c->h_est) (void)hipHostFree(c->h_est);
    if (c->h_norm) (void)hipHostFree(c->h_norm);
    if (c->h_kstate) (void)hipHostFree(c->h_kstate);
    c->h_est = c->h_norm = nullptr;
    c->h_kstate = nullptr;
    c->h_cap = 0;
  }
  const int64_t nch = (int64_t)c->chunk_inst.size();
  CHK(dalloc(c, &c->d_V, J * n * R));
  CHK(dalloc(c, &c->d_Z, restart * n * R));
  CHK(dalloc(c, &c->d_Wv, n * R));
  CHK(dalloc(c, &c->d_B, n * R));
  CHK(dalloc(c, &c->d_x, n * R));
  CHK(dalloc(c, &c->d_r, n * R));
  CHK(dalloc(c, &c->d_part, nch * J * R));
  CHK(dalloc(c, &c->d_part2, nch * J * R));
  CHK(dalloc(c, &c->d_npart, nch * R));
  CHK(dalloc(c, &c->d_h1, nsys * J));
  CHK(dalloc(c, &c->d_h2, nsys * J));
  CHK(dalloc(c, &c->d_Hs, nsys * J * J));
  CHK(dalloc(c, &c->d_cs, nsys * J));
  CHK(dalloc(c, &c->d_sn, nsys * J));
  CHK(dalloc(c, &c->d_g, nsys * J));
  CHK(dalloc(c, &c->d_hnorm, nsys));
  CHK(dalloc(c, &c->d_y, nsys * J));
  CHK(dalloc(c, &c->d_beta, nsys));
  CHK(dalloc(c, &c->d_kstate, 10 * nsys));
  c->kstate_n = nsys;
  c->d_jsys = reinterpret_cast<int32_t*>(c->d_kstate);
  c->d_its = reinterpret_cast<int32_t*>(c->d_kstate + 4 * nsys);
  c->d_active = c->d_kstate + 8 * nsys;
  c->d_mode = c->d_kstate + 9 * nsys;
  CHK(dalloc(c, &c->d_bnorm, nsys));
  CHK(dalloc(c, &c->d_nk, nsys));
  CHK(dalloc(c, &c->d_fin, nsys));
  if (!c->h_est) {
    HIPCHK(hipHostMalloc((void**)&c->h_est, 2 * nsys * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->h_norm, nsys * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->h_kstate, 10 * nsys, hipHostMallocDefault));
    c->h_cap = nsys;
  }
  for (hipEvent_t& e : c->ev_step)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipMemsetAsync(c->d_V, 0, J * n * R * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->d_Z, 0, restart * n * R * sizeof(double), c->stream));
  c->R_kry = R;
  c->restart_kry = restart;
  return MBDDC_OK;
}

template <int R>
int gmres_impl(mbddc_ctx* c, int nrhs, mbddc_info* info) {
  const Plan& P = c->plan;
  const int restart = c->opt.restart, J = restart + 1;
  const int64_t n = P.n_dofs;
  const int nsys = P.n_inst * R;
  const double rtol = c->opt.rtol;
  const int max_it = c->opt.max_it;
  KrylovArgs ka{};
  ka.chunk_inst = c->d_chunk_inst; ka.chunk_begin = c->d_chunk_begin; ka.inst_chunk_off = c->d_inst_chunk_off;
  ka.nchunks = (int32_t)c->chunk_inst.size(); ka.R = R; ka.jmax1 = J; ka.nrows = n;
  const unsigned nch = (unsigned)c->chunk_inst.size();
  const unsigned gv = nblk(n * R);
  const unsigned gs = nblk(nsys, 64);
  std::vector<int32_t> j(nsys, 0), its(nsys, 0), rest(nsys, 0), nk(nsys, 0);
  std::vector<uint8_t> active(nsys, 0), mode(nsys, 2), fin(nsys, 0), done(nsys, 0);
  std::vector<double> bnorm(nsys, 0.0), est(nsys, 0.0), rres(nsys, 0.0);
  auto h2d = [&](void* d, const void* h, size_t b) { return hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, c->stream); };
  // ||b||
  hipLaunchKernelGGL((k_residual<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_B, nullptr, nullptr, c->d_npart);
  hipLaunchKernelGGL(k_norms, dim3(nsys), dim3(64), 0, c->stream, ka, nsys, c->d_npart, c->h_norm);
  HIPCHK(hipMemsetAsync(c->d_x, 0, n * R * sizeof(double), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int s = 0; s < nsys; ++s) {
    bnorm[s] = c->h_norm[s];
    int k = s % R;
    if (k >= nrhs || bnorm[s] == 0.0) {
      done[s] = 1;
      continue;
    }
    active[s] = 1;
    fin[s] = 1;
    mode[s] = 0;
  }
  // r = b (x0 = 0): V_0 = b / ||b||, g = (||b||, 0, ...)
  HIPCHK(h2d(c->d_fin, fin.data(), nsys));
  HIPCHK(h2d(c->d_beta, bnorm.data(), nsys * sizeof(double)));
  HIPCHK(h2d(c->d_bnorm, bnorm.data(), nsys * sizeof(double)));
  hipLaunchKernelGGL((k_restart<R>), dim3(gv), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_B, c->d_fin, c->d_beta,
                     c->d_dof_inst);
  hipLaunchKernelGGL(k_restart_g, dim3(gs), dim3(64), 0, c->stream, ka, nsys, c->d_fin, c->d_beta, c->d_g);
  int status = MBDDC_OK;
  bool state_dirty = true;
  const GmresStop stop{c->d_its, c->d_mode, c->d_bnorm, rtol, restart, max_it};
  // One Arnoldi step of every system running on the device (CGS2, then the Givens step, which
  // writes the residual estimates into est_slot and advances or pauses each system).
  auto enqueue_step = [&](int jtop, double* est_slot) -> int {
    const double vbytes = 8.0 * n * R;                 // one block vector
    {
      ProfScope ps(c, F_KRYLOV_VEC, 2.0 * vbytes, 0.0);
      hipLaunchKernelGGL((k_next_vector<R>), dim3(gv), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_Wv, c->d_jsys,
                         c->d_mode, c->d_hnorm, c->d_dof_inst, c->d_X);
    }
    CHK(apply_run(c, R));
    {
      ProfScope ps(c, F_KRYLOV_VEC, 2.0 * vbytes, 0.0);
      hipLaunchKernelGGL((k_store_z<R>), dim3(gv), dim3(kBlock), 0, c->stream, ka, c->d_Y, c->d_Z, c->d_jsys,
                         c->d_active, c->d_dof_inst);
    }
    CHK(spmv_dispatch(c, R, c->d_Y, c->d_Wv));
    // CGS2
    const double jb = (jtop + 1) * vbytes, jf = 2.0 * (jtop + 1) * n * R;
    {
      ProfScope ps(c, F_KRYLOV_DOTS, jb + vbytes, jf);
      hipLaunchKernelGGL((k_dots<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_Wv, c->d_jsys,
                         c->d_active, jtop, c->d_part);
    }
    {
      ProfScope ps(c, F_KRYLOV_SMALL, 0.0, 0.0);
      hipLaunchKernelGGL(k_reduce_dots, dim3(nblk((int64_t)nsys * (jtop + 1), 4)), dim3(kBlock), 0, c->stream, ka,
                         c->d_part, nsys, jtop, c->d_h1);
    }
    {
      ProfScope ps(c, F_KRYLOV_UPDATE, jb + 2.0 * vbytes, jf);
      hipLaunchKernelGGL((k_update<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_Wv, c->d_h1,
                         c->d_jsys, c->d_active, c->d_dof_inst, jtop, (double*)nullptr);
    }
    {
      ProfScope ps(c, F_KRYLOV_DOTS, jb + vbytes, jf);
      hipLaunchKernelGGL((k_dots<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_Wv, c->d_jsys,
                         c->d_active, jtop, c->d_part2);
    }
    {
      ProfScope ps(c, F_KRYLOV_SMALL, 0.0, 0.0);
      hipLaunchKernelGGL(k_reduce_dots, dim3(nblk((int64_t)nsys * (jtop + 1), 4)), dim3(kBlock), 0, c->stream, ka,
                         c->d_part2, nsys, jtop, c->d_h2);
    }
    {
      ProfScope ps(c, F_KRYLOV_UPDATE, jb + 2.0 * vbytes, jf);
      hipLaunchKernelGGL((k_update<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_Wv, c->d_h2,
                         c->d_jsys, c->d_active, c->d_dof_inst, jtop, c->d_npart);
    }
    {
      ProfScope ps(c, F_KRYLOV_SMALL, 0.0, 0.0);
      hipLaunchKernelGGL(k_givens, dim3(nsys), dim3(64), 0, c->stream, ka, nsys, c->d_h1, c->d_h2, c->d_npart,
                         c->d_jsys, c->d_active, c->d_Hs, c->d_cs, c->d_sn, c->d_g, c->d_hnorm, est_slot, stop);
    }
    HIPCHK(hipGetLastError());
    return MBDDC_OK;
  };
  // The host's copy of the stop decision of every system that ran the step whose estimates are in
  // est_slot (the Givens step took the same decision on the device); systems that stop are marked
  // in fin (and paused on the device until the host has finished their cycle). fin is cleared
  // first unless it already holds the stops of the step before (both end their cycles together).
  std::vector<uint8_t> running(nsys, 0);
  std::vector<double> est_prev(nsys, 0.0);
  auto take_step = [&](const double* est_slot, bool clear_fin) {
    if (clear_fin) std::fill(fin.begin(), fin.end(), 0);
    bool any_fin = false;
    for (int s = 0; s < nsys; ++s) {
      if (!running[s]) continue;
      its[s]++;
      est_prev[s] = est[s];
      est[s] = est_slot[s];
      bool conv = est[s] <= rtol * bnorm[s];
      bool brk = !(est[s] == est[s]);
      if (conv || j[s] + 1 >= restart || its[s] >= max_it || brk) {
        fin[s] = 1;
        nk[s] = j[s] + 1;
        running[s] = 0;
        any_fin = true;
      } else {
        j[s]++;
        mode[s] = 1;
      }
    }
    return any_fin;
  };
  // Whether some running system will likely go on after its current step: not at the end of its
  // cycle or of its iteration budget, and not about to converge at its present rate.
  auto worth_next = [&](int& jnext) {
    bool any = false;
    jnext = 0;
    for (int s = 0; s < nsys; ++s) {
      if (!running[s] || j[s] + 1 >= restart || its[s] + 1 >= max_it) continue;
      jnext = std::max(jnext, j[s] + 1);
      const double e1 = est[s], e0 = est_prev[s];
      const bool soon = j[s] > 0 && e0 > 0.0 && e1 * (e1 / e0) <= 4.0 * rtol * bnorm[s];
      any |= !soon;
    }
    return any;
  };
  double* est_buf[2] = {c->h_est, c->h_est + c->kstate_n};
  int slot = 0;
  bool inflight = false;   // a step has been enqueued whose estimates the host has not taken yet
  while (true) {
    if (!inflight) {
      bool any = false;
      for (int s = 0; s < nsys; ++s) any |= active[s] != 0;
      if (!any) break;
      // the systems' state, in one copy, when the host has changed it (no step is in flight, so the
      // pinned buffer is free); otherwise the Givens step has advanced it on the device already
      if (state_dirty) {
        const int64_t kn = c->kstate_n;   // section offsets as allocated (a narrower solve uses a prefix)
        std::memcpy(c->h_kstate, j.data(), nsys * sizeof(int32_t));
        std::memcpy(c->h_kstate + 4 * kn, its.data(), nsys * sizeof(int32_t));
        std::memcpy(c->h_kstate + 8 * kn, active.data(), nsys);
        std::memcpy(c->h_kstate + 9 * kn, mode.data(), nsys);
        HIPCHK(h2d(c->d_kstate, c->h_kstate, 10 * kn));
        state_dirty = false;
      }
      int jtop = 0;
      for (int s = 0; s < nsys; ++s) {
        running[s] = active[s];
        if (active[s]) jtop = std::max(jtop, j[s]);
      }
      CHK(enqueue_step(jtop, est_buf[slot]));
      HIPCHK(hipEventRecord(c->ev_step[slot], c->stream));
      inflight = true;
    }
    // Enqueue the next step before the host waits for this one (the device advances the systems
    // that go on and pauses those that stop), so the host's wait and launches overlap the device.
    int jnext = 0;
    const bool ahead = worth_next(jnext);
    if (ahead) {
      CHK(enqueue_step(jnext, est_buf[slot ^ 1]));
      HIPCHK(hipEventRecord(c->ev_step[slot ^ 1], c->stream));
    }
    HIPCHK(hipEventSynchronize(c->ev_step[slot]));
    bool any_fin = take_step(est_buf[slot], true);
    slot ^= 1;
    inflight = ahead;
    if (!any_fin) continue;
    if (ahead) {   // finish the step already enqueued: its stops join this cycle's end
      HIPCHK(hipEventSynchronize(c->ev_step[slot]));
      take_step(est_buf[slot], false);
      slot ^= 1;
      inflight = false;
    }
    state_dirty = true;   // finished systems restart or leave: the host sends their state
    HIPCHK(h2d(c->d_fin, fin.data(), nsys));
    HIPCHK(h2d(c->d_nk, nk.data(), nsys * sizeof(int32_t)));
    hipLaunchKernelGGL(k_backsolve, dim3(gs), dim3(64), 0, c->stream, ka, nsys, c->d_fin, c->d_nk, c->d_Hs, c->d_g,
                       c->d_y);
    hipLaunchKernelGGL((k_xupdate<R>), dim3(gv), dim3(kBlock), 0, c->stream, ka, c->d_x, c->d_Z, c->d_y, c->d_fin,
                       c->d_nk, c->d_dof_inst);
    CHK(spmv_dispatch(c, R, c->d_x, c->d_Y));   // W of continuing systems stays intact
    hipLaunchKernelGGL((k_residual<R>), dim3(nch), dim3(kBlock), 0, c->stream, ka, c->d_B, c->d_Y, c->d_r, c->d_npart);
    hipLaunchKernelGGL(k_norms, dim3(nsys), dim3(64), 0, c->stream, ka, nsys, c->d_npart, c->h_norm);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<uint8_t> rs(nsys, 0);
    std::vector<double> beta(nsys, 0.0);
    bool any_rs = false;
    for (int s = 0; s < nsys; ++s) {
      if (!fin[s]) continue;
      rres[s] = c->h_norm[s];
      if (rres[s] <= rtol * bnorm[s]) {
        active[s] = 0;
        done[s] = 1;
      } else if (its[s] >= max_it || !(rres[s] == rres[s])) {
        active[s] = 0;
        done[s] = 2;
        status = MBDDC_ERR_NOCONV;
      } else {
        rs[s] = 1;
        beta[s] = rres[s];
        j[s] = 0;
        mode[s] = 0;
        rest[s]++;
        any_rs = true;
      }
    }
    if (any_rs) {
      HIPCHK(h2d(c->d_fin, rs.data(), nsys));
      HIPCHK(h2d(c->d_beta, beta.data(), nsys * sizeof(double)));
      hipLaunchKernelGGL((k_restart<R>), dim3(gv), dim3(kBlock), 0, c->stream, ka, c->d_V, c->d_r, c->d_fin,
                         c->d_beta, c->d_dof_inst);
      hipLaunchKernelGGL(k_restart_g, dim3(gs), dim3(64), 0, c->stream, ka, nsys, c->d_fin, c->d_beta, c->d_g);
    }
  }
  c->last_nrhs = nrhs;
  c->last_its.assign((size_t)c->plan.n_inst * nrhs, 0);
  for (int s = 0; s < nsys; ++s)
    if ((s % R) < nrhs) c->last_its[(size_t)(s / R) * nrhs + (s % R)] = its[s];
  if (info) {
    info->iterations = 0;
    info->restarts = 0;
    info->rel_res_true = 0.0;
    info->rel_res_est = 0.0;
    for (int s = 0; s < nsys; ++s) {
      if (bnorm[s] == 0.0 || (s % R) >= nrhs) continue;
      info->iterations = std::max(info->iterations, its[s]);
      info->restarts = std::max(info->restarts, rest[s]);
      info->rel_res_true = std::max(info->rel_res_true, rres[s] / bnorm[s]);
      info->rel_res_est = std::max(info->rel_res_est, est[s] / bnorm[s]);
    }
    info->status = status;
  }
  return status;
}

int gmres_dispatch(mbddc_ctx* c, int R, int nrhs, mbddc_info* info) {
  switch (R) {
    case 1: return gmres_impl<1>(c, nrhs, info);
    case 2: return gmres_impl<2>(c, nrhs, info);
    case 4: return gmres_impl<4>(c, nrhs, info);
    default: return gmres_impl<8>(c, nrhs, info);
  }
}

// ---------------------------------------------------------------------------
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device` (which is current), looked up once per device.
int scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return MBDDC_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return MBDDC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    last_hip_error() = e;
    return MBDDC_ERR_DEVICE;
  }
  g_scratch_ptr[device] = p;
  return MBDDC_OK;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// 1D tables of the Lagrange basis of order p (equispaced nodes on [0,1]) at the p+1 point
// Gauss-Legendre rule on [0,1].
ElemTables elem_tables(int order) {
  ElemTables t{};
  const int n = order + 1;
  double g[3], w[3];
  if (order == 1) {
    const double h = 0.5 / std::sqrt(3.0);
    g[0] = 0.5 - h; g[1] = 0.5 + h; w[0] = w[1] = 0.5;
  } else {
    const double h = 0.5 * std::sqrt(0.6);
    g[0] = 0.5 - h; g[1] = 0.5; g[2] = 0.5 + h;
    w[0] = w[2] = 5.0 / 18.0; w[1] = 8.0 / 18.0;
  }
  for (int q = 0; q < n; ++q) {
    const double x = g[q];
    t.w1[q] = w[q];
    if (order == 1) {
      t.N1[q][0] = 1.0 - x; t.N1[q][1] = x;
      t.D1[q][0] = -1.0; t.D1[q][1] = 1.0;
      t.Dend[q][0] = -1.0; t.Dend[q][1] = 1.0;   // q = end point 0 / 1 (n = 2 of them here)
    } else {
      t.N1[q][0] = 2.0 * (x - 0.5) * (x - 1.0); t.N1[q][1] = -4.0 * x * (x - 1.0); t.N1[q][2] = 2.0 * x * (x - 0.5);
      t.D1[q][0] = 4.0 * x - 3.0; t.D1[q][1] = -8.0 * x + 4.0; t.D1[q][2] = 4.0 * x - 1.0;
    }
  }
  if (order == 2) {
    t.Dend[0][0] = -3.0; t.Dend[0][1] = 4.0; t.Dend[0][2] = -1.0;
    t.Dend[1][0] = 1.0; t.Dend[1][1] = -4.0; t.Dend[1][2] = 3.0;
  }
  return t;
}

// Element tangents (and element forces when fe) at the displacement in d_u, into d_Ke.
int launch_elements(mbddc_ctx* c, bool forces) {
  ElemArgs g{};
  g.coords = c->d_coords; g.u = c->d_u; g.elem_nodes = c->d_elem_nodes; g.node_off = c->d_elem_node_off;
  g.ke_off = c->d_ke_off; g.elem_mat = c->d_elem_mat; g.mats = c->d_mats; g.frames = c->d_frames;
  g.Ke = c->d_Ke; g.fe = forces ? c->d_fe : nullptr; g.fe_off = c->d_fe_off; g.flag = c->d_flag;
  for (int o = 0; o < 2; ++o) {
    if (c->el_list[o].empty()) continue;
    g.elems = c->d_el_list[o];
    g.n = (int64_t)c->el_list[o].size();
    const ElemTables tab = elem_tables(o + 1);
    ProfScope ps(c, F_ELEMENT, 8.0 * (c->plan.ke_total), 0.0);
    if (o == 0) hipLaunchKernelGGL((k_element<2>), dim3((unsigned)g.n), dim3(kBlock), 0, c->stream, g, tab);
    else hipLaunchKernelGGL((k_element<3>), dim3((unsigned)g.n), dim3(kBlock), 0, c->stream, g, tab);
  }
  for (int o = 0; o < 2; ++o) {   // boundary faces, added to their elements' matrices and forces
    if (c->bc_end[o].empty()) continue;
    FaceArgs f{};
    f.coords = c->d_coords; f.u = c->d_u; f.elem_nodes = c->d_elem_nodes; f.node_off = c->d_elem_node_off;
    f.ke_off = c->d_ke_off; f.fe_off = c->d_fe_off; f.items = c->d_bc_items[o]; f.item_end = c->d_bc_end[o];
    f.faces = c->d_faces; f.bcs = c->d_bcs; f.n = (int64_t)c->bc_end[o].size(); f.Ke = c->d_Ke;
    f.fe = forces ? c->d_fe : nullptr; f.flag = c->d_flag;
    const ElemTables tab = elem_tables(o + 1);
    ProfScope ps(c, F_ELEMENT, 0.0, 0.0);
    if (o == 0) hipLaunchKernelGGL((k_element_faces<2>), dim3((unsigned)f.n), dim3(kBlock), 0, c->stream, f, tab);
    else hipLaunchKernelGGL((k_element_faces<3>), dim3((unsigned)f.n), dim3(kBlock), 0, c->stream, f, tab);
  }
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

// The assembled operator from the element matrices in d_Ke.
int assemble_operator(mbddc_ctx* c) {
  {
    ProfScope ps(c, F_ASSEMBLE_BSR, c->op_bytes[F_ASSEMBLE_BSR], 0.0);
    hipLaunchKernelGGL(k_assemble_bsr, dim3(nblk(c->nblocks * 9)), dim3(kBlock), 0, c->stream, c->d_Ke, c->d_bsr_rowptr,
                       c->d_bsr_rownode, c->d_bsr_col, c->d_bsr_cptr, c->d_bsr_contrib, c->d_bsr_kstride, c->d_free,
                       c->nblocks, c->d_vals);
  }
  HIPCHK(hipGetLastError());
  return MBDDC_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* mbddc_strerror(int status) {
  switch (status) {
    case MBDDC_OK: return "ok";
    case MBDDC_ERR_ARG: return "invalid argument";
    case MBDDC_ERR_OOM: return "device out of memory";
    case MBDDC_ERR_SINGULAR: return "singular local or coarse problem";
    case MBDDC_ERR_NOCONV: return "GMRES did not converge";
    case MBDDC_ERR_DEVICE: return "HIP runtime error";
    case MBDDC_ERR_STATE: return "call out of order";
    case MBDDC_ERR_UNSUPPORTED: return "unsupported size or option";
    default: return "unknown status";
  }
}

int mbddc_default_options(mbddc_options* opt) {
  if (!opt) return MBDDC_ERR_ARG;
  std::memset(opt, 0, sizeof(*opt));
  opt->primal = MBDDC_PRIMAL_V | MBDDC_PRIMAL_E;
  opt->levels = 2;
  opt->coarse_group = 8;
  opt->coarse_primal = MBDDC_PRIMAL_V | MBDDC_PRIMAL_E | MBDDC_PRIMAL_F;
  opt->precision = MBDDC_MIXED;
  opt->restart = 30;
  opt->rtol = 1e-8;
  opt->max_it = 1000;
  opt->graph_apply = 1;
  opt->packed_sym = 1;
  opt->nonsym_coarse = 1;
  return MBDDC_OK;
}

int mbddc_create(mbddc_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return MBDDC_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MBDDC_ERR_DEVICE;
  if (hip_device < 0 || hip_device >= ndev) return MBDDC_ERR_ARG;
  if (hipSetDevice(hip_device) != hipSuccess) return MBDDC_ERR_DEVICE;
  CHK(scratch_init(hip_device));   // the no-allocation entry point's buffer on this device
  mbddc_ctx* c = new (std::nothrow) mbddc_ctx();
  if (!c) return MBDDC_ERR_OOM;
  c->device = hip_device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  mbddc_default_options(&c->opt);
  *out = c;
  return MBDDC_OK;
}

int mbddc_release(mbddc_ctx* c) {
  if (!c) return MBDDC_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  else HIPCHK(hipDeviceSynchronize());
  release_buffers(c);
  c->state = 0;
  c->R_alloc = 0; c->R_kry = 0; c->restart_kry = 0; c->Y_R = 0;
  c->last_its.clear();
  c->last_nrhs = 0;
  return MBDDC_OK;
}

int mbddc_destroy(mbddc_ctx* c) {
  if (!c) return MBDDC_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_all(c);
  delete c;
  return MBDDC_OK;
}

}  // extern "C"

namespace {
int parse_meshes(int n_inst, const mbddc_mesh* meshes, const mbddc_options* opt, mbddc_options& o,
                 std::vector<MeshIn>& ms) {
  if (n_inst <= 0 || !meshes) return MBDDC_ERR_ARG;
  if (opt) o = *opt;
  else mbddc_default_options(&o);
  if ((o.levels != 2 && o.levels != 3) || o.coarse_group < 1 || (o.coarse_primal & ~7u) || o.restart < 1 || o.restart > 63 || !(o.rtol > 0.0) || o.max_it < 1 ||
      (o.precision != MBDDC_FP64 && o.precision != MBDDC_MIXED && o.precision != MBDDC_MIXED_F32FACT) ||
      (o.primal & ~7u) || (o.nnsp != 0 && o.nnsp != 1) ||
      (o.scaling != MBDDC_SCALING_COUNTING && o.scaling != MBDDC_SCALING_DELUXE))
    return MBDDC_ERR_ARG;
  // deluxe scaling: symmetric path with FP64 local factors
  if (o.scaling == MBDDC_SCALING_DELUXE && (o.symmetric_hint == 0 || o.precision == MBDDC_MIXED_F32FACT))
    return MBDDC_ERR_UNSUPPORTED;
  if (o.nnsp && o.levels == 3) return MBDDC_ERR_UNSUPPORTED;   // level-2 nodes carry three components
  ms.assign(n_inst, MeshIn());
  for (int i = 0; i < n_inst; ++i) {
    const mbddc_mesh& m = meshes[i];
    if (m.n_nodes <= 0 || m.n_elems <= 0 || m.n_sub <= 0 || !m.elem_nodes || !m.elem_part ||
        (m.n_dirichlet > 0 && !m.dirichlet_dofs) || m.n_dirichlet < 0)
      return MBDDC_ERR_ARG;
    int npe = m.elem_type == MBDDC_HEX8 ? 8 : (m.elem_type == MBDDC_HEX27 ? 27 : 0);
    if (!npe) return MBDDC_ERR_ARG;
    MeshIn& mi = ms[i];
    mi.n_nodes = m.n_nodes; mi.n_elems = m.n_elems; mi.npe = npe; mi.n_sub = m.n_sub;
    mi.elem_nodes.assign(m.elem_nodes, m.elem_nodes + (int64_t)m.n_elems * npe);
    mi.elem_part.assign(m.elem_part, m.elem_part + m.n_elems);
    if (m.node_tags) mi.node_tags.assign(m.node_tags, m.node_tags + m.n_nodes);
    if (m.n_dirichlet > 0) mi.dirichlet.assign(m.dirichlet_dofs, m.dirichlet_dofs + m.n_dirichlet);
    if (m.coords) {
      for (int64_t k = 0; k < 3LL * m.n_nodes; ++k)
        if (!std::isfinite(m.coords[k])) return MBDDC_ERR_ARG;
      mi.coords.assign(m.coords, m.coords + 3LL * m.n_nodes);
    }
  }
  return MBDDC_OK;
}

// Host part of the symbolic setup: plan, layout and (three levels) the level-2 plan.
// Reads a tuning table written by mbddc_autotune (the format is documented in mbddc.h).
int read_tuning(const char* path, Tuning& t) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return MBDDC_ERR_ARG;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < (1u << 20)) text.append(buf, k);
  std::fclose(f);
  if (text.find("\"mbddc_tune\"") == std::string::npos) return MBDDC_ERR_ARG;
  auto ints_after = [&](const char* key, int32_t* out, int n) -> bool {
    size_t p = text.find(key);
    if (p == std::string::npos) return false;
    p = text.find(':', p);
    if (p == std::string::npos) return false;
    const char* q = text.c_str() + p + 1;
    for (int i = 0; i < n; ++i) {
      while (*q == ' ' || *q == '\t' || *q == '\n' || *q == '\r' || *q == '[' || (i > 0 && *q == ',')) ++q;
      char* e = nullptr;
      const long v = std::strtol(q, &e, 10);
      if (e == q) return false;
      out[i] = (int32_t)v;
      q = e;
    }
    return true;
  };
  Tuning r;
  if (!ints_after("\"sym_fp64\"", r.sym[0], kSymBuckets) || !ints_after("\"sym_fp32\"", r.sym[1], kSymBuckets) ||
      !ints_after("\"apply_xchunk\"", &r.xchunk, 1))
    return MBDDC_ERR_ARG;
  if (text.find("\"apply_groups\"") != std::string::npos) {
    if (!ints_after("\"apply_groups\"", &r.apply_big, 1) || r.apply_big < -1 || r.apply_big > 1) return MBDDC_ERR_ARG;
  }
  if (text.find("\"gemm_mfma\"") != std::string::npos) {
    if (!ints_after("\"gemm_mfma\"", &r.gemm_mfma, 1) || (r.gemm_mfma != 0 && r.gemm_mfma != 1)) return MBDDC_ERR_ARG;
  }
  if (text.find("\"apply_rows\"") != std::string::npos) {
    if (!ints_after("\"apply_rows\"", r.apply_rows, 4)) return MBDDC_ERR_ARG;
    for (int k = 0; k < 4; ++k)
      if (r.apply_rows[k] != 0 && r.apply_rows[k] != 64 && r.apply_rows[k] != 128 && r.apply_rows[k] != 256)
        return MBDDC_ERR_ARG;
  }
  if (text.find("\"apply_rows2\"") != std::string::npos) {
    if (!ints_after("\"apply_rows2\"", r.apply_rows2, 4)) return MBDDC_ERR_ARG;
    for (int k = 0; k < 4; ++k)
      if (r.apply_rows2[k] != 0 && r.apply_rows2[k] != 64 && r.apply_rows2[k] != 128 && r.apply_rows2[k] != 256)
        return MBDDC_ERR_ARG;
  }
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < kSymBuckets; ++b)
      if (r.sym[p][b] < 0 || r.sym[p][b] >= SV_COUNT) return MBDDC_ERR_ARG;
  if (r.xchunk < 64 || r.xchunk > kApplyChunk || r.xchunk % 64) return MBDDC_ERR_ARG;
  t = r;
  return MBDDC_OK;
}

int prepare_host(mbddc_ctx* c, const mbddc_options& o, const std::vector<MeshIn>& ms) {
  c->tune = Tuning();
  if (o.tune_table) CHK(read_tuning(o.tune_table, c->tune));
  c->opt = o;
  c->opt.tune_table = nullptr;   // read once; the caller's string is not kept
  c->mixed = (o.precision != MBDDC_FP64);
  c->fact32 = (o.precision == MBDDC_MIXED_F32FACT);
  c->sym = (o.symmetric_hint != 0);
  c->deluxe = (o.scaling == MBDDC_SCALING_DELUXE);
  std::string err = build_plan(ms, o.primal, c->plan, o.nnsp != 0);
  if (!err.empty()) return MBDDC_ERR_ARG;
  c->h_tags.clear();
  for (const MeshIn& m : ms) {
    if (m.node_tags.empty()) c->h_tags.insert(c->h_tags.end(), m.n_nodes, 0u);
    else c->h_tags.insert(c->h_tags.end(), m.node_tags.begin(), m.node_tags.end());
  }
  c->h_coords.clear();
  bool all_coords = true;
  for (const MeshIn& m : ms) all_coords &= !m.coords.empty();
  if (all_coords)
    for (const MeshIn& m : ms) c->h_coords.insert(c->h_coords.end(), m.coords.begin(), m.coords.end());
  CHK(build_layout(c));
  if (o.levels == 3) CHK(build_level2_host(c, ms));
  return MBDDC_OK;
}

int factor_dispatch(mbddc_ctx* c) {
  c->last_bad = 0;
  return c->fact32 ? factor_impl<float, float>(c)
                   : (c->mixed ? factor_impl<double, float>(c) : factor_impl<double, double>(c));
}

// Regroups the symmetric inversions and the apply row blocks after a change of c->tune
// (and the level-2 child's).
int rebuild_symsets(mbddc_ctx* c) {
  if (c->sym) {
    for (SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
      dfree(c, S->d_all); dfree(c, S->d_big); dfree(c, S->d_items); dfree(c, S->d_gd); dfree(c, S->d_gitems);
    }
    if (!(c->set_kii.build(c->gj_kii, c->fact32, c->tune) && c->set_x.build(c->gj_x, c->fact32, c->tune) &&
          c->set_t.build(c->gj_t, c->fact32, c->tune) && c->set_dlx.build(c->gj_dlx, false, c->tune)))
      return MBDDC_ERR_UNSUPPORTED;
    for (SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
      CHK(upload(c, &S->d_all, S->all));
      CHK(upload(c, &S->d_big, S->big));
      CHK(upload(c, &S->d_items, S->items));
      CHK(upload(c, &S->d_gd, S->gd));
      CHK(upload(c, &S->d_gitems, S->gitems));
    }
    int64_t pb = 0, bc = 0;
    for (const SymSet* S : {&c->set_kii, &c->set_x, &c->set_t, &c->set_dlx}) {
      pb = std::max(pb, S->pbuf_elems);
      bc = std::max(bc, (int64_t)S->big.size());
    }
    if (pb > c->big_pbuf || bc > c->big_count || (bc > 0 && !c->d_bpanel)) {
      dfree(c, c->d_bpanel); dfree(c, c->d_bdinv); dfree(c, c->d_bthr);
      c->big_pbuf = std::max(pb, c->big_pbuf);
      c->big_count = std::max(bc, c->big_count);
      CHK(dalloc(c, &c->d_bpanel, c->big_pbuf));
      CHK(dalloc(c, &c->d_bdinv, c->big_count * kSymCB * kSymCB));
      CHK(dalloc(c, &c->d_bthr, c->big_count));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  // apply row blocks
  dfree(c, c->d_itA); dfree(c, c->d_itC); dfree(c, c->d_itF); dfree(c, c->d_itH);
  build_apply_items(c);
  CHK(upload(c, &c->d_itA, c->itA));
  CHK(upload(c, &c->d_itC, c->itC));
  CHK(upload(c, &c->d_itF, c->itF));
  CHK(upload(c, &c->d_itH, c->itH));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->apply_gen++;                 // staging width and row blocks are baked into the captured applies
  if (c->child) {
    c->child->tune = child_tuning(c->tune);
    CHK(rebuild_symsets(c->child));
  }
  return MBDDC_OK;
}

// GPU time (ms) of fn() on the handle's stream, best of `reps`.
template <typename F>
int time_best(mbddc_ctx* c, int reps, F fn, double* best) {
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  *best = 1e300;
  int st = MBDDC_OK;
  for (int r = 0; r < reps && st == MBDDC_OK; ++r) {
    (void)hipEventRecord(a, c->stream);
    st = fn();
    (void)hipEventRecord(b, c->stream);
    if (hipEventSynchronize(b) != hipSuccess) st = MBDDC_ERR_DEVICE;
    float ms = 0.0f;
    if (st == MBDDC_OK && hipEventElapsedTime(&ms, a, b) == hipSuccess) *best = std::min(*best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

// Coordinate search over the tuning table on this handle's own matrices: for each size
// bucket that occurs in the symmetric inversions, every variant that can take the
// bucket's matrices is timed by a whole numeric factorisation (best of two); then the
// apply staging width by the apply of four right-hand sides (best of five). The handle
// ends factorised with the chosen table.
int autotune_impl(mbddc_ctx* c) {
  const int p = c->fact32 ? 1 : 0;
  if (c->sym) {
    int bmax[kSymBuckets] = {0, 0, 0, 0};
    for (const std::vector<GjDesc>* v : {&c->gj_kii, &c->gj_x, &c->gj_t})
      for (const GjDesc& g : *v)
        if (g.n > 0) bmax[sym_bucket(g.n)] = std::max(bmax[sym_bucket(g.n)], g.n);
    for (int b = 0; b < kSymBuckets; ++b) {
      if (bmax[b] == 0) continue;
      int best_v = c->tune.sym[p][b];
      double best_t = 1e300;
      for (int v = 0; v < SV_COUNT; ++v) {
        if (!sym_variant_ok(v, bmax[b], p == 1)) continue;
        c->tune.sym[p][b] = v;
        CHK(rebuild_symsets(c));
        double t = 0.0;
        CHK(time_best(c, 2, [&] { return factor_dispatch(c); }, &t));
        if (t < best_t) {
          best_t = t;
          best_v = v;
        }
      }
      c->tune.sym[p][b] = best_v;
      CHK(rebuild_symsets(c));
    }
  }
  {   // batched GEMMs: vector units or matrix cores
    int best_g = c->tune.gemm_mfma;
    double best_t = 1e300;
    for (int g = 0; g < 2; ++g) {
      c->tune.gemm_mfma = g;
      if (c->child) c->child->tune.gemm_mfma = g;
      double t = 0.0;
      CHK(time_best(c, 2, [&] { return factor_dispatch(c); }, &t));
      if (t < best_t) {
        best_t = t;
        best_g = g;
      }
    }
    c->tune.gemm_mfma = best_g;
    if (c->child) c->child->tune.gemm_mfma = best_g;
  }
  CHK(factor_dispatch(c));
  // apply staging width
  CHK(ensure_apply_buffers(c, 4));
  hipLaunchKernelGGL(k_fill, dim3(nblk(c->plan.n_dofs * 4)), dim3(kBlock), 0, c->stream, c->d_X,
                     c->plan.n_dofs * 4, 0.0);
  int best_x = c->tune.xchunk;
  double best_t = 1e300;
  const int top = std::min(kApplyChunk, (int)round_up(std::max(c->max_cols, 1), 64));
  for (int xc : {128, 256, 512, 1024}) {
    if (xc > top && xc != 128) continue;
    c->tune.xchunk = xc;
    if (c->child) c->child->tune.xchunk = xc;
    CHK(apply_dispatch(c, 4, c->d_X, c->d_Y));
    double t = 0.0;
    CHK(time_best(c, 5, [&] { return apply_dispatch(c, 4, c->d_X, c->d_Y); }, &t));
    if (t < best_t) {
      best_t = t;
      best_x = xc;
    }
  }
  c->tune.xchunk = best_x;
  if (c->child) c->child->tune.xchunk = best_x;
  {   // apply column groups of the local phases
    int best_g = 0;
    best_t = 1e300;
    for (int g : {0, 1}) {
      c->tune.apply_big = g;
      CHK(rebuild_symsets(c));
      CHK(apply_dispatch(c, 4, c->d_X, c->d_Y));
      double t = 0.0;
      CHK(time_best(c, 5, [&] { return apply_dispatch(c, 4, c->d_X, c->d_Y); }, &t));
      if (t < best_t) {
        best_t = t;
        best_g = g;
      }
    }
    c->tune.apply_big = best_g;
  }
  // rows per workgroup of each local apply phase
  for (int k = 0; k < 4; ++k) {
    int best_r = c->apply_rows_eff[k];
    best_t = 1e300;
    for (int rw : {256, 128, 64}) {
      c->tune.apply_rows[k] = rw;
      CHK(rebuild_symsets(c));
      CHK(apply_dispatch(c, 4, c->d_X, c->d_Y));
      double t = 0.0;
      CHK(time_best(c, 5, [&] { return apply_dispatch(c, 4, c->d_X, c->d_Y); }, &t));
      if (t < best_t) {
        best_t = t;
        best_r = rw;
      }
    }
    c->tune.apply_rows[k] = best_r;
  }
  // rows per workgroup of the level-2 apply phases
  for (int k = 0; k < 4 && c->child; ++k) {
    int best_r = c->child->apply_rows_eff[k];
    best_t = 1e300;
    for (int rw : {256, 128, 64}) {
      c->tune.apply_rows2[k] = rw;
      CHK(rebuild_symsets(c));
      CHK(apply_dispatch(c, 4, c->d_X, c->d_Y));
      double t = 0.0;
      CHK(time_best(c, 5, [&] { return apply_dispatch(c, 4, c->d_X, c->d_Y); }, &t));
      if (t < best_t) {
        best_t = t;
        best_r = rw;
      }
    }
    c->tune.apply_rows2[k] = best_r;
  }
  CHK(rebuild_symsets(c));
  return MBDDC_OK;
}
}  // namespace

extern "C" {

int mbddc_estimate_footprint(int n_inst, const mbddc_mesh* meshes, const mbddc_options* opt, int nrhs,
                             size_t* device_bytes) {
  if (!device_bytes || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  mbddc_options o;
  std::vector<MeshIn> ms;
  int st = parse_meshes(n_inst, meshes, opt, o, ms);
  if (st) return st;
  mbddc_ctx tmp;   // host only: no device call is made on it
  st = prepare_host(&tmp, o, ms);
  if (!st) *device_bytes = (size_t)device_bytes_estimate(&tmp, true, nrhs);
  if (tmp.child) {
    delete tmp.child;
    tmp.child = nullptr;
  }
  return st;
}

int mbddc_setup_symbolic_batch(mbddc_ctx* c, int n_inst, const mbddc_mesh* meshes, const mbddc_options* opt) {
  if (!c || n_inst <= 0 || !meshes) return MBDDC_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  mbddc_options o;
  std::vector<MeshIn> ms;
  CHK(parse_meshes(n_inst, meshes, opt, o, ms));
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  release_buffers(c);
  c->subs.clear();
  c->last_its.clear();
  c->last_nrhs = 0;
  c->R_alloc = 0; c->R_kry = 0; c->restart_kry = 0; c->Y_R = 0;
  c->d_tb = c->d_wb = c->d_cc = nullptr;
  c->d_ep = c->d_X = c->d_Y = c->d_io = nullptr;
  c->d_V = c->d_Z = c->d_Wv = c->d_B = c->d_x = c->d_r = nullptr;
  c->d_part = c->d_part2 = c->d_npart = c->d_h1 = c->d_h2 = c->d_Hs = c->d_cs = c->d_sn = c->d_g = nullptr;
  c->d_hnorm = c->d_y = c->d_beta = nullptr;
  c->d_jsys = c->d_nk = c->d_its = nullptr;
  c->d_active = c->d_mode = c->d_fin = c->d_kstate = nullptr;
  c->d_bnorm = nullptr;
  c->d_Kc_keep = nullptr;
  c->d_cDinv = c->d_cY = c->d_cCcol = nullptr;
  c->d_csym_gd = nullptr;
  c->d_csym_items = nullptr;
  c->d_l2_eidx = nullptr;
  c->d_l2_inv = nullptr;
  c->state = 0;
  int st = prepare_host(c, o, ms);
  if (!st) st = upload_plan(c);
  if (!st && c->child) st = upload_level2(c);
  if (!st) st = dalloc(c, &c->d_flag, 1);
  if (!st && !c->h_flag) st = hipHostMalloc((void**)&c->h_flag, sizeof(int32_t), hipHostMallocDefault) == hipSuccess
                                  ? MBDDC_OK : MBDDC_ERR_DEVICE;
  if (st) {
    release_buffers(c);
    return st;
  }
  c->state = 1;
  return MBDDC_OK;
}

int mbddc_setup_symbolic(mbddc_ctx* c, const mbddc_mesh* mesh, const mbddc_options* opt) {
  return mbddc_setup_symbolic_batch(c, 1, mesh, opt);
}

int mbddc_footprint(const mbddc_ctx* c, int nrhs, size_t* device_bytes) {
  if (!c || !device_bytes || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  const Plan& P = c->plan;
  const int R = apply_R(nrhs), J = c->opt.restart + 1;
  // per-call buffers that a solve with nrhs right-hand sides allocates, unless already held
  size_t extra = 0;
  if (c->R_alloc < R) {
    extra += (size_t)P.n_slots * R * 8 * 2 + (size_t)std::max<int64_t>(P.n_cslots, 1) * R * 8;
    extra += (size_t)c->nchunk_max * std::max<int64_t>(P.n_coarse, 1) * R * 8 + (size_t)P.n_dofs * R * 8 * 3;
    if (c->packed) extra += (size_t)(c->np_total + c->tp_total) * R * 8;
  }
  if (c->R_kry < R || c->restart_kry < c->opt.restart) extra += (size_t)P.n_dofs * R * 8 * (2 * J + 4);
  if (const mbddc_ctx* ch = c->child) {   // level-2 operators and its apply buffers
    const Plan& Q = ch->plan;
    extra += ch->bytes;
    if (ch->R_alloc < R) {
      extra += (size_t)Q.n_slots * R * 8 * 2 + (size_t)std::max<int64_t>(Q.n_cslots, 1) * R * 8;
      extra += (size_t)ch->nchunk_max * std::max<int64_t>(Q.n_coarse, 1) * R * 8 + (size_t)Q.n_dofs * R * 8 * 3;
      if (ch->packed) extra += (size_t)(ch->np_total + ch->tp_total) * R * 8;
    }
  }
  *device_bytes = c->bytes + extra;
  return MBDDC_OK;
}

int mbddc_get_sizes(const mbddc_ctx* c, mbddc_sizes* out) {
  if (!c || !out) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  const Plan& P = c->plan;
  out->n_dofs = P.n_dofs;
  out->n_free = P.n_free;
  out->n_interface = P.n_ifx;
  out->n_coarse = P.n_coarse;
  out->n_sub = P.n_sub;
  out->n_instances = P.n_inst;
  out->n_vertices = P.n_vertices;
  out->n_edges = P.n_edges;
  out->n_faces = P.n_faces;
  out->max_local = P.max_local;
  out->bsr_blocks = c->nblocks;
  out->n_sub2 = c->child ? c->child->plan.n_sub : 0;
  out->n_coarse2 = c->child ? c->child->plan.n_coarse : 0;
  return MBDDC_OK;
}

int mbddc_set_tangent(mbddc_ctx* c, const double* elem_K, int on_device) {
  if (!c || !elem_K) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const Plan& P = c->plan;
  HIPCHK(hipMemcpyAsync(c->d_Ke, elem_K, P.ke_total * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  // reject NaN / Inf before the operator is touched (one read of K_e on the device)
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::min<int64_t>(4096, nblk(P.ke_total))), dim3(kBlock), 0,
                     c->stream, c->d_Ke, P.ke_total, c->d_flag);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (*c->h_flag) {   // operator and factors untouched; the element matrices must be set again
    c->ke_valid = false;
    return MBDDC_ERR_ARG;
  }
  c->ke_valid = true;
  {
    ProfScope ps(c, F_ASSEMBLE_BSR, c->op_bytes[F_ASSEMBLE_BSR], 0.0);
    hipLaunchKernelGGL(k_assemble_bsr, dim3(nblk(c->nblocks * 9)), dim3(kBlock), 0, c->stream, c->d_Ke, c->d_bsr_rowptr,
                       c->d_bsr_rownode, c->d_bsr_col, c->d_bsr_cptr, c->d_bsr_contrib, c->d_bsr_kstride, c->d_free,
                       c->nblocks, c->d_vals);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->state = std::max(c->state, 2);
  return MBDDC_OK;
}

int mbddc_set_material(mbddc_ctx* c, const mbddc_material* mats, const double* frames) {
  if (!c || !mats) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const Plan& P = c->plan;
  if ((int64_t)c->h_coords.size() != 3 * P.n_nodes) return MBDDC_ERR_ARG;   // meshes came without coordinates
  std::vector<MatDev> md(P.n_inst);
  bool guccione = false;
  for (int i = 0; i < P.n_inst; ++i) {
    const mbddc_material& m = mats[i];
    if (m.kind != MBDDC_MAT_SVK && m.kind != MBDDC_MAT_NEO_HOOKEAN && m.kind != MBDDC_MAT_GUCCIONE) return MBDDC_ERR_ARG;
    md[i].kind = m.kind;
    for (int k = 0; k < 6; ++k) {
      if (!std::isfinite(m.p[k])) return MBDDC_ERR_ARG;
      md[i].p[k] = m.p[k];
    }
    guccione |= m.kind == MBDDC_MAT_GUCCIONE;
  }
  if (guccione && !frames) return MBDDC_ERR_ARG;
  for (int o = 0; o < 2; ++o) { c->bc_items[o].clear(); c->bc_end[o].clear(); }   // conditions set again after
  std::vector<int32_t> elem_mat(P.n_elems);
  for (int i = 0; i < P.n_inst; ++i)
    for (int32_t e = 0; e < P.inst[i].n_elems; ++e) elem_mat[P.inst[i].elem_off + e] = i;
  for (int o = 0; o < 2; ++o) c->el_list[o].clear();
  std::vector<int64_t> fe_off(P.n_elems + 1, 0);
  for (int64_t e = 0; e < P.n_elems; ++e) {
    const int npe = P.elem_npe[e];
    if (npe != 8 && npe != 27) return MBDDC_ERR_UNSUPPORTED;
    c->el_list[npe == 8 ? 0 : 1].push_back((int32_t)e);
    fe_off[e + 1] = fe_off[e] + 3 * npe;
  }
  // node -> (element force entry) in ascending element order: the fixed order of the force gather
  std::vector<int32_t> ne_ptr(P.n_nodes + 1, 0);
  for (int64_t e = 0; e < P.n_elems; ++e)
    for (int a = 0; a < P.elem_npe[e]; ++a) ne_ptr[P.elem_nodes_flat[P.elem_node_off[e] + a] + 1]++;
  for (int64_t n = 0; n < P.n_nodes; ++n) ne_ptr[n + 1] += ne_ptr[n];
  std::vector<int64_t> ne_ent(ne_ptr[P.n_nodes]);
  std::vector<int32_t> fill(ne_ptr.begin(), ne_ptr.end() - 1);
  for (int64_t e = 0; e < P.n_elems; ++e)
    for (int a = 0; a < P.elem_npe[e]; ++a) ne_ent[fill[P.elem_nodes_flat[P.elem_node_off[e] + a]]++] = fe_off[e] + 3 * a;
  for (auto* p : {&c->d_coords, &c->d_u, &c->d_frames, &c->d_fe, &c->d_fint}) dfree(c, *p);
  dfree(c, c->d_elem_nodes); dfree(c, c->d_elem_node_off); dfree(c, c->d_elem_mat); dfree(c, c->d_mats);
  dfree(c, c->d_el_list[0]); dfree(c, c->d_el_list[1]); dfree(c, c->d_fe_off); dfree(c, c->d_ne_ptr);
  dfree(c, c->d_ne_ent);
  c->have_material = false;
  CHK(upload(c, &c->d_coords, c->h_coords));
  CHK(dalloc(c, &c->d_u, P.n_dofs));
  CHK(dalloc(c, &c->d_fe, fe_off[P.n_elems]));
  CHK(dalloc(c, &c->d_fint, P.n_dofs));
  CHK(upload(c, &c->d_elem_nodes, P.elem_nodes_flat));
  CHK(upload(c, &c->d_elem_node_off, P.elem_node_off));
  CHK(upload(c, &c->d_elem_mat, elem_mat));
  CHK(upload(c, &c->d_mats, md));
  for (int o = 0; o < 2; ++o) CHK(upload(c, &c->d_el_list[o], c->el_list[o]));
  CHK(upload(c, &c->d_fe_off, fe_off));
  CHK(upload(c, &c->d_ne_ptr, ne_ptr));
  CHK(upload(c, &c->d_ne_ent, ne_ent));
  if (guccione) {
    std::vector<double> fr(frames, frames + 9 * P.n_elems);
    for (double v : fr)
      if (!std::isfinite(v)) return MBDDC_ERR_ARG;
    CHK(upload(c, &c->d_frames, fr));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  c->have_material = true;
  return MBDDC_OK;
}

int mbddc_set_boundary(mbddc_ctx* c, const mbddc_boundary* bcs, int n_bc) {
  if (!c || n_bc < 0 || (n_bc > 0 && !bcs)) return MBDDC_ERR_ARG;
  if (c->state < 1 || !c->have_material) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const Plan& P = c->plan;
  std::vector<BcDev> bd(n_bc);
  for (int b = 0; b < n_bc; ++b) {
    const mbddc_boundary& x = bcs[b];
    if ((x.kind != MBDDC_BC_ROBIN && x.kind != MBDDC_BC_PRESSURE) || x.tag == 0 || x.instance < -1 ||
        x.instance >= P.n_inst || !std::isfinite(x.p[0]) || !std::isfinite(x.p[1]))
      return MBDDC_ERR_ARG;
    bd[b].kind = x.kind;
    bd[b].p[0] = x.p[0];
    bd[b].p[1] = x.p[1];
  }
  // faces xi_d = side of every element whose nodes all carry a condition's tag bits
  std::vector<int32_t> faces;
  for (int o = 0; o < 2; ++o) { c->bc_items[o].clear(); c->bc_end[o].clear(); }
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const Instance& in = P.inst[ii];
    for (int32_t el = 0; el < in.n_elems; ++el) {
      const int64_t e = in.elem_off + el;
      const int npe = P.elem_npe[e], p1 = npe == 8 ? 2 : 3;
      const int32_t first = (int32_t)(faces.size() / 3);
      for (int b = 0; b < n_bc; ++b) {
        if (bcs[b].instance >= 0 && bcs[b].instance != ii) continue;
        for (int d = 0; d < 3; ++d)
          for (int side = 0; side < 2; ++side) {
            bool on = true;
            for (int a = 0; a < npe && on; ++a) {
              const int ia[3] = {a % p1, (a / p1) % p1, a / (p1 * p1)};
              if (ia[d] != side * (p1 - 1)) continue;
              on = (c->h_tags[P.elem_nodes_flat[P.elem_node_off[e] + a]] & bcs[b].tag) == bcs[b].tag;
            }
            if (on) faces.insert(faces.end(), {d, side, b});
          }
      }
      const int32_t last = (int32_t)(faces.size() / 3);
      if (last > first) {
        const int o = npe == 8 ? 0 : 1;
        c->bc_items[o].insert(c->bc_items[o].end(), {(int32_t)e, first});
        c->bc_end[o].push_back(last);
      }
    }
  }
  for (int o = 0; o < 2; ++o) { dfree(c, c->d_bc_items[o]); dfree(c, c->d_bc_end[o]); }
  dfree(c, c->d_faces);
  dfree(c, c->d_bcs);
  for (int o = 0; o < 2; ++o) {
    CHK(upload(c, &c->d_bc_items[o], c->bc_items[o]));
    CHK(upload(c, &c->d_bc_end[o], c->bc_end[o]));
  }
  CHK(upload(c, &c->d_faces, faces));
  CHK(upload(c, &c->d_bcs, bd));
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

int mbddc_set_displacement(mbddc_ctx* c, const double* u, int on_device, double* f_int, int f_on_device) {
  if (!c || !u) return MBDDC_ERR_ARG;
  if (c->state < 1 || !c->have_material) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const Plan& P = c->plan;
  HIPCHK(hipMemcpyAsync(c->d_u, u, P.n_dofs * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
  CHK(launch_elements(c, f_int != nullptr));
  HIPCHK(hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (*c->h_flag) {   // the element matrices are invalid: the operator and factors stay as they were
    c->ke_valid = false;
    return MBDDC_ERR_ARG;
  }
  CHK(assemble_operator(c));
  c->ke_valid = true;
  if (f_int) {
    hipLaunchKernelGGL(k_gather_forces, dim3(nblk(3 * P.n_nodes)), dim3(kBlock), 0, c->stream, c->d_ne_ptr, c->d_ne_ent,
                       c->d_fe, c->d_free, P.n_nodes, c->d_fint);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(f_int, c->d_fint, P.n_dofs * sizeof(double),
                          f_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  c->state = std::max(c->state, 2);
  return MBDDC_OK;
}

int mbddc_get_element_tangents(const mbddc_ctx* c, double* Ke, int on_device) {
  if (!c || !Ke) return MBDDC_ERR_ARG;
  if (c->state < 2) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  HIPCHK(hipMemcpyAsync(Ke, c->d_Ke, c->plan.ke_total * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

int mbddc_factor(mbddc_ctx* c) {
  if (!c) return MBDDC_ERR_ARG;
  if (c->state < 2 || !c->ke_valid) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  int st = factor_dispatch(c);
  if (st != MBDDC_OK) {
    c->state = 2;
    return st;
  }
  c->state = 3;
  return MBDDC_OK;
}

int mbddc_autotune(mbddc_ctx* c, const char* table_out) {
  if (!c) return MBDDC_ERR_ARG;
  if (c->state < 2) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const uint32_t mask = c->prof.mask;
  c->prof.mask = 0;
  int st = autotune_impl(c);
  c->prof.mask = mask;
  if (st != MBDDC_OK) {
    c->state = 2;
    return st;
  }
  c->state = 3;
  if (table_out) {
    FILE* f = std::fopen(table_out, "wb");
    if (!f) return MBDDC_ERR_ARG;
    const Tuning& t = c->tune;
    std::fprintf(f,
                 "{\"mbddc_tune\": 1,\n \"variants\": [\"%s\", \"%s\", \"%s\", \"%s\"],\n"
                 " \"bucket_max_n\": [%d, %d, %d, null],\n"
                 " \"sym_fp64\": [%d, %d, %d, %d],\n \"sym_fp32\": [%d, %d, %d, %d],\n"
                 " \"apply_xchunk\": %d,\n \"apply_rows\": [%d, %d, %d, %d],\n"
                 " \"apply_rows2\": [%d, %d, %d, %d],\n \"apply_groups\": %d,\n \"gemm_mfma\": %d}\n",
                 kSymVariantName[0], kSymVariantName[1], kSymVariantName[2], kSymVariantName[3], kSymBucketMax[0],
                 kSymBucketMax[1], kSymBucketMax[2], t.sym[0][0], t.sym[0][1], t.sym[0][2], t.sym[0][3], t.sym[1][0],
                 t.sym[1][1], t.sym[1][2], t.sym[1][3], t.xchunk, c->apply_rows_eff[0], c->apply_rows_eff[1],
                 c->apply_rows_eff[2], c->apply_rows_eff[3], t.apply_rows2[0], t.apply_rows2[1], t.apply_rows2[2],
                 t.apply_rows2[3], t.apply_big, t.gemm_mfma);
    const bool bad = std::ferror(f) != 0;
    if (std::fclose(f) != 0 || bad) return MBDDC_ERR_ARG;
  }
  return MBDDC_OK;
}

int mbddc_get_tuning(const mbddc_ctx* c, int32_t* sym_fp64, int32_t* sym_fp32, int32_t* apply_xchunk,
                     int32_t* apply_rows, int32_t* gemm_mfma) {
  if (!c) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  for (int b = 0; b < kSymBuckets; ++b) {
    if (sym_fp64) sym_fp64[b] = c->tune.sym[0][b];
    if (sym_fp32) sym_fp32[b] = c->tune.sym[1][b];
  }
  if (apply_xchunk) *apply_xchunk = c->tune.xchunk;
  for (int k = 0; k < 4 && apply_rows; ++k) apply_rows[k] = c->apply_rows_eff[k];
  if (gemm_mfma) *gemm_mfma = c->tune.gemm_mfma;
  return MBDDC_OK;
}

int mbddc_apply(mbddc_ctx* c, int nrhs, const double* r, double* z, int on_device) {
  if (!c || !r || !z || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  if (c->state < 3) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const int R = apply_R(nrhs);
  CHK(ensure_apply_buffers(c, R));
  CHK(load_block(c, r, nrhs, R, on_device, c->d_X));
  CHK(apply_run(c, R));
  return store_block(c, c->d_Y, nrhs, R, on_device, z);
}

int mbddc_matvec(mbddc_ctx* c, int nrhs, const double* x, double* y, int on_device) {
  if (!c || !x || !y || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  if (c->state < 2) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  const int R = apply_R(nrhs);
  CHK(ensure_apply_buffers(c, R));
  CHK(load_block(c, x, nrhs, R, on_device, c->d_X));
  CHK(spmv_dispatch(c, R, c->d_X, c->d_Y));
  return store_block(c, c->d_Y, nrhs, R, on_device, y);
}

int mbddc_matvec_noalloc(mbddc_ctx* c, int nrhs, const double* x, double* y) {
  if (!c || !x || !y || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  const int R = apply_R(nrhs);
  const int64_t n = c->plan.n_dofs;
  const size_t blk = (size_t)round_up(n * R * (int64_t)sizeof(double), 256);
  if (2 * blk > kScratchBytes) return MBDDC_ERR_UNSUPPORTED;   // beyond the static buffer
  if (c->state < 2) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(c->device));
  if (!base) return MBDDC_ERR_STATE;
  double* X = reinterpret_cast<double*>(base);
  double* Y = reinterpret_cast<double*>(base + blk);
  // every entry of X (zeros past nrhs and on clamped DOFs) and of Y is written below, so the
  // buffer needs no clearing between calls
  hipLaunchKernelGGL(k_to_interleaved, dim3(nblk(n * R)), dim3(kBlock), 0, c->stream, x, nrhs, R, n, c->d_free, X);
  if (c->nblocks > kSpmvWideRow * c->plan.n_nodes)
    launch_spmv<64>(c, R, X, Y);
  else
    launch_spmv<32>(c, R, X, Y);
  hipLaunchKernelGGL(k_from_interleaved, dim3(nblk(n * nrhs)), dim3(kBlock), 0, c->stream, Y, nrhs, R, n, y);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return MBDDC_OK;
}

int mbddc_solve(mbddc_ctx* c, int nrhs, const double* b, double* x, int on_device, mbddc_info* info) {
  if (!c || !b || !x || nrhs < 1 || nrhs > kMaxRhs) return MBDDC_ERR_ARG;
  if (c->state < 3) return MBDDC_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  double t0 = now_ms();
  const int R = apply_R(nrhs);
  CHK(ensure_apply_buffers(c, R));
  CHK(ensure_krylov(c, R));
  CHK(load_block(c, b, nrhs, R, on_device, c->d_B));
  c->n_applies = c->n_applies_graphed = 0;
  int st = gmres_dispatch(c, R, nrhs, info);
  int st2 = store_block(c, c->d_x, nrhs, R, on_device, x);
  if (info) {
    info->ms_solve = now_ms() - t0;
    info->bad_subdomain = 0;
    info->applies = c->n_applies;
    info->applies_graphed = c->n_applies_graphed;
  }
  return st != MBDDC_OK ? st : st2;
}

int mbddc_get_globs(const mbddc_ctx* c, int32_t* node_glob, int32_t* n_globs, int32_t* glob_kind,
                    int32_t* coarse_glob, int32_t* coarse_comp) {
  if (!c) return MBDDC_ERR_ARG;
  if (c->state < 1) return MBDDC_ERR_STATE;
  const Plan& P = c->plan;
  if (node_glob) std::copy(P.node_glob.begin(), P.node_glob.end(), node_glob);
  if (n_globs) *n_globs = (int32_t)P.glob_kind.size();
  if (glob_kind) std::copy(P.glob_kind.begin(), P.glob_kind.end(), glob_kind);
  if (coarse_glob) std::copy(P.coarse_glob.begin(), P.coarse_glob.end(), coarse_glob);
  if (coarse_comp) std::copy(P.coarse_comp.begin(), P.coarse_comp.end(), coarse_comp);
  return MBDDC_OK;
}

int mbddc_get_coarse_matrix(const mbddc_ctx* c, int inst, double* out, int64_t n_c) {
  if (!c || !out || inst < 0) return MBDDC_ERR_ARG;
  if (c->state < 3 || !c->d_Kc_keep) return MBDDC_ERR_STATE;
  if (inst >= c->plan.n_inst || n_c != c->inst_nc[inst]) return MBDDC_ERR_ARG;
  const int ld = c->inst_kc_ld[inst];
  std::vector<double> t((size_t)ld * std::max<int64_t>(n_c, 1));
  if (hipMemcpy(t.data(), c->d_Kc_keep + c->inst_kc_off[inst], t.size() * sizeof(double), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return MBDDC_ERR_DEVICE;
  for (int64_t k = 0; k < n_c; ++k)
    for (int64_t l = 0; l < n_c; ++l) out[l * n_c + k] = t[(size_t)k * ld + l];   // stored transposed
  return MBDDC_OK;
}

int mbddc_get_bsr(const mbddc_ctx* c, int32_t* rowptr, int32_t* colidx, double* vals) {
  if (!c) return MBDDC_ERR_ARG;
  if (c->state < 2) return MBDDC_ERR_STATE;
  const Plan& P = c->plan;
  if (rowptr) std::copy(P.bsr_rowptr.begin(), P.bsr_rowptr.end(), rowptr);
  if (colidx) std::copy(P.bsr_col.begin(), P.bsr_col.end(), colidx);
  if (vals) {
    std::vector<double> v(c->nblocks * 9);
    if (hipMemcpy(v.data(), c->d_vals, v.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return MBDDC_ERR_DEVICE;
    for (int64_t n = 0; n < P.n_nodes; ++n) {
      int32_t r0 = P.bsr_rowptr[n], nb = P.bsr_rowptr[n + 1] - r0;
      for (int32_t j = 0; j < nb; ++j)
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q)
            vals[9LL * (r0 + j) + 3 * p + q] = v[9LL * r0 + (int64_t)p * 3 * nb + 3LL * j + q];
    }
  }
  return MBDDC_OK;
}

int mbddc_last_bad_subdomain(const mbddc_ctx* c) { return c ? c->last_bad : 0; }

int mbddc_get_iterations(const mbddc_ctx* c, int32_t* its, int64_t max_entries, int64_t* n_entries) {
  if (!c || (!its && max_entries > 0)) return MBDDC_ERR_ARG;
  if (c->state < 3) return MBDDC_ERR_STATE;
  const int64_t n = (int64_t)c->last_its.size();
  if (n_entries) *n_entries = n;
  for (int64_t k = 0; k < std::min(n, max_entries); ++k) its[k] = c->last_its[k];
  return MBDDC_OK;
}

int mbddc_set_allocator(mbddc_ctx* c, void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* user) {
  if (!c || (!alloc) != (!free_)) return MBDDC_ERR_ARG;
  if (c->state != 0 || !c->allocs.empty()) return MBDDC_ERR_STATE;
  c->alloc_fn = alloc;
  c->free_fn = free_;
  c->alloc_user = alloc ? user : nullptr;
  return MBDDC_OK;
}

const char* mbddc_profile_family_name(int family) {
  return (family >= 0 && family < F_COUNT) ? kFamilyName[family] : nullptr;
}

int mbddc_set_profiling(mbddc_ctx* c, uint32_t family_mask) {
  if (!c) return MBDDC_ERR_ARG;
  c->prof.mask = family_mask;
  return MBDDC_OK;
}

int mbddc_get_profile(mbddc_ctx* c, mbddc_kernel_stat* out, int max_entries, int* n_entries) {
  if (!c || (max_entries > 0 && !out)) return MBDDC_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return MBDDC_ERR_DEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MBDDC_ERR_DEVICE;
  Profiler& p = c->prof;
  for (auto& e : p.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) p.ms[e.fam] += ms;
    p.pool.push_back(e.a);
    p.pool.push_back(e.b);
  }
  p.pending.clear();
  int k = 0;
  for (int f = 0; f < F_COUNT; ++f) {
    if (p.launches[f] == 0) continue;
    if (k < max_entries) {
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kFamilyName[f]);
      out[k].launches = p.launches[f];
      out[k].ms = p.ms[f];
      out[k].bytes = p.bytes[f];
      out[k].flops = p.flops[f];
    }
    ++k;
    p.launches[f] = 0;
    p.ms[f] = p.bytes[f] = p.flops[f] = 0.0;
  }
  if (n_entries) *n_entries = k;
  return MBDDC_OK;
}

int mbddc_inspect_symbolic(const mbddc_mesh* m, uint32_t primal, mbddc_sizes* sizes, int32_t* node_glob,
                           int32_t* glob_kind, int32_t* coarse_glob, int32_t* coarse_comp, int32_t* sub_counts) {
  if (!m || (primal & ~7u)) return MBDDC_ERR_ARG;
  int npe = m->elem_type == MBDDC_HEX8 ? 8 : (m->elem_type == MBDDC_HEX27 ? 27 : 0);
  if (!npe || m->n_nodes <= 0 || m->n_elems <= 0 || m->n_sub <= 0 || !m->elem_nodes || !m->elem_part ||
      m->n_dirichlet < 0 || (m->n_dirichlet > 0 && !m->dirichlet_dofs))
    return MBDDC_ERR_ARG;
  std::vector<MeshIn> ms(1);
  MeshIn& mi = ms[0];
  mi.n_nodes = m->n_nodes; mi.n_elems = m->n_elems; mi.npe = npe; mi.n_sub = m->n_sub;
  mi.elem_nodes.assign(m->elem_nodes, m->elem_nodes + (int64_t)m->n_elems * npe);
  mi.elem_part.assign(m->elem_part, m->elem_part + m->n_elems);
  if (m->node_tags) mi.node_tags.assign(m->node_tags, m->node_tags + m->n_nodes);
  if (m->n_dirichlet > 0) mi.dirichlet.assign(m->dirichlet_dofs, m->dirichlet_dofs + m->n_dirichlet);
  Plan P;
  if (!build_plan(ms, primal, P).empty()) return MBDDC_ERR_ARG;
  if (sizes) {
    sizes->n_dofs = P.n_dofs; sizes->n_free = P.n_free; sizes->n_interface = P.n_ifx; sizes->n_coarse = P.n_coarse;
    sizes->n_sub = P.n_sub; sizes->n_instances = 1; sizes->n_vertices = P.n_vertices; sizes->n_edges = P.n_edges;
    sizes->n_faces = P.n_faces; sizes->max_local = P.max_local; sizes->bsr_blocks = (int64_t)P.bsr_col.size();
  }
  if (node_glob) std::copy(P.node_glob.begin(), P.node_glob.end(), node_glob);
  if (glob_kind) std::copy(P.glob_kind.begin(), P.glob_kind.end(), glob_kind);
  if (coarse_glob) std::copy(P.coarse_glob.begin(), P.coarse_glob.end(), coarse_glob);
  if (coarse_comp) std::copy(P.coarse_comp.begin(), P.coarse_comp.end(), coarse_comp);
  if (sub_counts)
    for (int64_t s = 0; s < P.n_sub; ++s) {
      sub_counts[3 * s] = P.subs[s].nI;
      sub_counts[3 * s + 1] = P.subs[s].nG;
      sub_counts[3 * s + 2] = P.subs[s].nc;
    }
  return MBDDC_OK;
}

}  // extern "C"
