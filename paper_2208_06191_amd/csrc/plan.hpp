// Host-side symbolic setup of the BDDC decomposition (paper §3.2, §4).
//
// Everything here is integer work done once per mesh: DOF maps, interface
// multiplicity, vertex/edge/face globs, primal constraint rows, coarse
// numbering, the assembled 3x3-block pattern and the per-subdomain dense
// layouts that the device kernels use. No floating-point arithmetic of the
// method happens here (constraint weights 1/m and counting weights
// 1/|N(x)| are the only reals produced).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mbddc {

enum GlobKind { kVertex = 1, kEdge = 2, kFace = 4 };

struct MeshIn {
  int32_t n_nodes = 0;
  int32_t n_elems = 0;
  int32_t npe = 0;         // 8 or 27 (fixed-size elements)
  int32_t n_sub = 0;
  std::vector<int32_t> elem_ptr;  // optional [n_elems+1]: variable-size elements (coarse levels)
  std::vector<int32_t> elem_nodes;
  std::vector<int32_t> elem_part;
  std::vector<uint32_t> node_tags;
  std::vector<int32_t> dirichlet;
  std::vector<double> coords;     // optional [n_nodes*3] (element kernels on the device)
};

// One subdomain's layout. Local DOFs are ordered interior first then interface,
// each ascending in global DOF id. All offsets are element counts into the
// corresponding concatenated arrays.
struct SubLayout {
  int32_t inst = 0;
  int32_t nI = 0, nG = 0, nc = 0;     // interior, interface, local primal constraints
  int32_t ni() const { return nI + nG; }
  int32_t mP() const { return nG + nc; } // size of the constrained interface problem
  int64_t dof_off = 0;                // into sub_dofs (ni entries: global DOF ids)
  int64_t if_off = 0;                 // first interface slot id (nG consecutive slots)
  int64_t c_off = 0;                  // first coarse slot id (nc consecutive slots)
  int64_t elem_off = 0;               // into sub_elems / elem_ldof (by element count)
  int32_t n_elems = 0;
  int64_t cons_off = 0;               // into cons_ptr (nc + 1 entries)
};

struct Instance {
  int32_t npe = 0;
  int64_t node_off = 0, elem_off = 0, sub_off = 0, coarse_off = 0, glob_off = 0;
  int32_t n_nodes = 0, n_elems = 0, n_sub = 0, n_coarse = 0, n_globs = 0;
  int64_t ke_off = 0;                 // first element-matrix entry of this instance
};

struct Plan {
  int32_t n_inst = 0;
  std::vector<Instance> inst;
  int64_t n_nodes = 0, n_dofs = 0, n_elems = 0, n_sub = 0, n_coarse = 0, n_free = 0;
  int64_t ke_total = 0;               // total entries of the element-matrix array
  std::vector<int64_t> ke_off;        // per element: first entry in the element-matrix array
  std::vector<int32_t> elem_npe;      // per element
  std::vector<int32_t> elem_nodes_flat; // global node ids, concatenated (npe per element)
  std::vector<int64_t> elem_node_off; // per element: offset into elem_nodes_flat
  std::vector<uint8_t> free_dof;      // [n_dofs]
  std::vector<int32_t> dof_inst;      // [n_dofs] instance of each DOF (used for vector segments)

  // globs (global numbering across instances, sorted per instance by first node)
  std::vector<int32_t> glob_kind;
  std::vector<int32_t> glob_node0;    // first (lowest) global node of each glob
  std::vector<int32_t> node_glob;     // [n_nodes] or -1
  std::vector<int32_t> coarse_glob, coarse_comp;   // [n_coarse] glob; component (row index for nnsp globs)
  int64_t n_vertices = 0, n_edges = 0, n_faces = 0;

  // assembled operator: 3x3 blocks over nodes
  std::vector<int32_t> bsr_rowptr, bsr_col;
  std::vector<int32_t> bsr_cptr;      // [blocks+1] into bsr_contrib
  std::vector<int64_t> bsr_contrib;   // element-matrix entry of the block's (0,0)
  std::vector<int32_t> bsr_kstride;   // [blocks] row stride (3 npe) of the contributing element matrices

  // subdomains
  std::vector<SubLayout> subs;
  std::vector<int32_t> sub_dofs;      // global DOF ids, per subdomain local order
  std::vector<int32_t> sub_elems;     // element ids per subdomain
  std::vector<int32_t> elem_ldof;     // per subdomain element: 3*npe local ids (-1: clamped)
  std::vector<int64_t> elem_ldof_off; // per subdomain element: offset into elem_ldof
  // constraint rows, local coarse order: entries (interface-local index, weight)
  std::vector<int32_t> cons_ptr;      // concatenated per subdomain, nc+1 each
  std::vector<int32_t> cons_idx;
  std::vector<double> cons_w;
  // interface slots
  int64_t n_slots = 0;
  std::vector<int32_t> slot_dof;      // [n_slots] global DOF
  std::vector<int32_t> slot_ifx;      // [n_slots] global interface index
  std::vector<double> slot_w;         // [n_slots] counting weight 1/|N(x)|
  std::vector<uint8_t> slot_owner;    // [n_slots] first slot of its interface DOF
  int64_t n_ifx = 0;
  std::vector<int32_t> ifx_ptr, ifx_slots;  // interface DOF -> slots (ascending subdomain)
  // coarse slots
  int64_t n_cslots = 0;
  std::vector<int32_t> cslot_coarse;  // [n_cslots] global coarse id
  std::vector<int32_t> coarse_ptr, coarse_slots; // coarse id -> slots (ascending subdomain)
  int64_t max_local = 0;
};

// Builds the plan for a batch of instances. Returns an empty string on success,
// an error message otherwise.
// With nnsp, primal edges and faces carry near-null-space rows (their rigid motions) instead of
// component averages; coarse_comp is then the row's index in the glob's basis.
std::string build_plan(const std::vector<MeshIn>& meshes, uint32_t primal, Plan& out, bool nnsp = false);

}  // namespace mbddc
