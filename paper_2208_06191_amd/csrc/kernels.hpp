// Device data layouts and kernel launchers of the BDDC hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbddc {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxRhs = 8;           // right-hand sides handled per call
constexpr int kGjMax = 512;          // largest matrix of the one-workgroup Gauss-Jordan kernel
constexpr int kCoarseBlock = 64;     // diagonal block of the multi-workgroup coarse inversion
constexpr int kCoarseChunk = 256;    // columns per workgroup in the coarse product
constexpr int kApplyChunk = 1024;    // input columns staged in LDS at a time by the local apply
constexpr int kApplyBigCols = 512;   // local blocks this wide take the large column groups (by size)
constexpr int kSpmvWideRow = 40;     // mean blocks per node row above which a node row takes 64 lanes

// Per-subdomain device descriptor. Offsets are element counts into the
// per-precision work buffers. Dense work matrices are row-major; apply
// operators are column-major with a leading dimension padded to 4.
struct SubDev {
  int32_t nI, nG, nc, inst;
  int32_t n_elems, ldK;               // ldK = nI + nG
  int64_t dof_off, if_off, c_off, elem_off, cons_off;
  int64_t oK;                         // K^(i) (ni x ni); its top-left nI block becomes K_II^-1
  int64_t oG;                         // K_GI K_II^-1   (nG x nI)
  int64_t oH;                         // K_II^-1 K_IG   (nI x nG)
  int64_t oP;                         // [S C^T; C 0] (mP x mP), inverted in place
  int64_t oB1, oB2, oB3, oB4;         // operators: [K_II^-1; G] (G alone when packed), [D S~ D; (D Phi)^T],
                                      // D Phi, H (-1 when packed)
  int32_t ld1, ld2, ld3, ld4;
  int64_t oKc;                        // local coarse matrix (nc x nc, FP64)
  int64_t oPiv;                       // pivots: nI for K_II then mP for P
  // Symmetric path, packed: K_II^-1 (slot 0) and [D S~ D; (D Phi)^T] (slot 1) with their symmetric
  // block stored once, as column panels of kSymPanel columns from the panel's diagonal row down
  // (SymPack below); -1 when stored full (oB1 / oB2). oNP / oTP: the partial products (units of
  // R-vectors) of the normal and transposed tile products.
  int64_t oS[2], oNP[2], oTP[2];
  // Packed path: phase A forms G r_I alone and phase H solves z_I = K_II^-1 (r_I - K_IG z_G), with
  // K_IG as CSR rows over the interior: row pointers (nI + 1, relative) at kig_ptr of the pointer
  // array, interface-local columns at kig_col of the column array, values at oKig of the operator
  // buffer (-1 otherwise).
  int64_t oKig, kig_ptr, kig_col;
  // Packed path, phase A: G (column-major, ld1 rows, ld1 a multiple of 32) applied by 256 x 256
  // tiles; their partial products per column panel at oNPA (panels(nI) x nG R-vectors).
  int64_t oNPA;
};

// Panel-packed symmetric operator: rows [0, n) = [S; X] with S (nS x nS) symmetric, columns
// [0, nS). Column panel p holds columns [kSymPanel p, kSymPanel (p + 1)) and rows [kSymPanel p, n)
// column-major with leading dimension N32 - kSymPanel p (N32 = n rounded up to 32, so every
// column segment of a row tile starts on a 128-byte boundary in FP32); the diagonal tile of a
// panel is stored whole. Panels are consecutive.
constexpr int kSymPanel = 256;
struct SymPack {
  __host__ __device__ static int32_t n32(int32_t n) { return (n + 31) / 32 * 32; }
  __host__ __device__ static int32_t panels(int32_t nS) { return (nS + kSymPanel - 1) / kSymPanel; }
  // first element of panel p; also the first partial row of panel p divided by kSymPanel
  __host__ __device__ static int64_t panel_rows_before(int32_t p, int32_t N32) {
    return (int64_t)p * N32 - (int64_t)(kSymPanel / 2) * p * (p - 1);
  }
  __host__ __device__ static int64_t panel_off(int32_t p, int32_t N32) {
    return (int64_t)kSymPanel * panel_rows_before(p, N32);
  }
  __host__ __device__ static int32_t ld(int32_t p, int32_t N32) { return N32 - kSymPanel * p; }
  __host__ __device__ static int64_t elems(int32_t nS, int32_t n) {
    const int32_t P = panels(nS), N32 = n32(n);
    if (P == 0) return 0;
    return panel_off(P - 1, N32) + (int64_t)(nS - kSymPanel * (P - 1)) * ld(P - 1, N32);
  }
  // rows of the normal partial products (all panels)
  __host__ __device__ static int64_t np_rows(int32_t nS, int32_t n) {
    const int32_t P = panels(nS), N32 = n32(n);
    return P == 0 ? 0 : panel_rows_before(P - 1, N32) + ld(P - 1, N32);
  }
  // transposed partial of panel b from row tile k (b < k < P), in units of kSymPanel entries
  __host__ __device__ static int64_t tp_index(int32_t b, int32_t k, int32_t P) {
    return (int64_t)b * (P - 1) - (int64_t)b * (b - 1) / 2 + (k - b - 1);
  }
  __host__ __device__ static int64_t tp_count(int32_t P) { return (int64_t)P * (P - 1) / 2; }
};

// Batched Gauss-Jordan descriptor: invert the n x n matrix at base+off (row stride ld).
struct GjDesc {
  int64_t off;
  int32_t n, ld;
  int64_t piv_off;
  int32_t id;                          // reported in the status array on a zero pivot
  int32_t pad;
};

// Large symmetric matrix of the batched blocked sweep: base + off, n x n, row stride ld
// (lower triangle used); panel buffers W and U (n x 128 each, U after W) at pbuf + pw.
struct BigSym {
  int64_t off, pw;
  int32_t n, ld;
  int32_t stat;                        // status slot
  int32_t pad;
};

// Batched GEMM descriptor: C = alpha * A B + beta * Ci (row-major, sizes M x K, K x N).
struct GemmDesc {
  int32_t M, N, K, lda, ldb, ldc, ldci, tiles_n;
  int64_t oA, oB, oC, oCi;
  double alpha, beta;
  int32_t transB, pad;                 // transB: B(k, n) is stored at B[n * ldb + k]
};

struct GemmItem {
  int32_t prob, tm, tn, pad;
};

// Deluxe scaling: one block per (subdomain, glob of its interface): the glob's n entries at
// idx[idx_off ..] (interface-local, ascending DOF), its n x n blocks S_g^(i) and D_g^(i) at off of
// their buffers, and the glob's summed block at toff.
struct DlxBlock {
  int64_t off, idx_off, toff;
  int32_t n, sub;
};
// A glob shared for deluxe scaling: its summed block (n x n) at toff, its blocks at
// gblk[first .. first + count) (ascending subdomain).
struct DlxGlob {
  int64_t toff;
  int32_t n, first, count, pad;
};

// Sparse products of the symmetric factorisation: up to kCgW consecutive interface columns
// [h0, h0 + nh) of one subdomain with the union of their K_IG patterns (nu interior rows, ascending,
// at row_off of the row array).
constexpr int kCgW = 16;
constexpr int kCgMaxRows = 768;
struct ColGroup {
  int64_t row_off;
  int32_t sub, h0, nh, nu;
};

// Workgroups are handed to the 8 XCDs round-robin; renumbering them so that each XCD takes one
// contiguous range of work items keeps the data those items share (a GEMM's panels, a sweep's
// panels, a SpMV row range's neighbourhood of x) in that XCD's L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned g) {
  const unsigned x = b % 8, i = b / 8, q = g / 8, r = g % 8;
  return x * q + min(x, r) + i;
}

// Apply work item: (subdomain or instance, first row, first column, column count).
struct ApplyItem {
  int32_t sub, row0, col0, ncol;
};

}  // namespace mbddc
