// Host-side symbolic setup: paper §3.2 index sets and §4 preallocation.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

namespace mbddc {
namespace {

struct UnionFind {
  std::vector<int32_t> p;
  explicit UnionFind(int32_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int32_t find(int32_t x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

int popcount32(uint32_t v) { return __builtin_popcount(v); }

// Near-null-space rows of one glob (paper §4, rigid motions as primal degrees of freedom): an
// orthonormal basis of the six rigid motions restricted to the glob's free DOFs. Candidates in
// the order translations x, y, z, rotations about x, y, z through the centroid of the glob's
// nodes; modified Gram-Schmidt with one re-orthogonalisation pass; a candidate left with at most
// 1e-8 of its norm is dependent and dropped. `dofs` receives the free DOFs (node-major, global
// ids), `rows` the r rows over them (row-major); returns r.
int rigid_rows(const MeshIn& m, const std::vector<int32_t>& nodes, const std::vector<uint8_t>& free_dof,
               int64_t node_off, std::vector<int32_t>& dofs, std::vector<double>& rows) {
  double cen[3] = {0.0, 0.0, 0.0};
  for (int32_t n : nodes)
    for (int a = 0; a < 3; ++a) cen[a] += m.coords[3 * (int64_t)n + a];
  for (int a = 0; a < 3; ++a) cen[a] /= (double)nodes.size();
  std::vector<double> dx;   // d = x - centroid per free DOF's node, and the DOF's component
  std::vector<int> comp;
  dofs.clear();
  for (int32_t n : nodes)
    for (int c = 0; c < 3; ++c) {
      const int64_t d = 3 * (node_off + n) + c;
      if (!free_dof[d]) continue;
      dofs.push_back((int32_t)d);
      comp.push_back(c);
      for (int a = 0; a < 3; ++a) dx.push_back(m.coords[3 * (int64_t)n + a] - cen[a]);
    }
  const size_t nd = dofs.size();
  std::vector<std::vector<double>> Q;
  std::vector<double> v(nd);
  for (int k = 0; k < 6; ++k) {
    for (size_t j = 0; j < nd; ++j) {
      const int c = comp[j];
      const double* d = &dx[3 * j];
      if (k < 3) {
        v[j] = (c == k) ? 1.0 : 0.0;
      } else {   // (e_a x d)_c for a = k - 3
        const int a = k - 3;
        const int c1 = (a + 1) % 3, c2 = (a + 2) % 3;   // e_a x d = (.., -d_c2 at c1, d_c1 at c2)
        v[j] = (c == c1) ? -d[c2] : (c == c2 ? d[c1] : 0.0);
      }
    }
    double n0 = 0.0;
    for (double x : v) n0 += x * x;
    n0 = std::sqrt(n0);
    if (n0 == 0.0) continue;
    for (int pass = 0; pass < 2; ++pass)
      for (const std::vector<double>& q : Q) {
        double dot = 0.0;
        for (size_t j = 0; j < nd; ++j) dot += q[j] * v[j];
        for (size_t j = 0; j < nd; ++j) v[j] -= dot * q[j];
      }
    double n1 = 0.0;
    for (double x : v) n1 += x * x;
    n1 = std::sqrt(n1);
    if (n1 <= 1e-8 * n0) continue;
    for (double& x : v) x /= n1;
    Q.push_back(v);
  }
  rows.clear();
  for (const std::vector<double>& q : Q) rows.insert(rows.end(), q.begin(), q.end());
  return (int)Q.size();
}

}  // namespace

std::string build_plan(const std::vector<MeshIn>& meshes, uint32_t primal, Plan& P, bool nnsp) {
  P = Plan();
  P.n_inst = static_cast<int32_t>(meshes.size());
  if (P.n_inst <= 0) return "no instance";
  // ---------------------------------------------------------------- offsets
  auto npe_of = [](const MeshIn& m, int32_t e) {
    return m.elem_ptr.empty() ? m.npe : m.elem_ptr[e + 1] - m.elem_ptr[e];
  };
  auto node_of = [](const MeshIn& m, int32_t e, int32_t a) {
    return m.elem_ptr.empty() ? m.elem_nodes[(int64_t)e * m.npe + a] : m.elem_nodes[m.elem_ptr[e] + a];
  };
  for (const MeshIn& m : meshes) {
    if (m.n_nodes <= 0 || m.n_elems <= 0 || m.n_sub <= 0) return "empty mesh or partition";
    if (m.elem_ptr.empty()) {
      if (m.npe != 8 && m.npe != 27) return "element type must be HEX8 or HEX27";
      if ((int64_t)m.elem_nodes.size() != (int64_t)m.n_elems * m.npe) return "elem_nodes size";
    } else {
      if ((int64_t)m.elem_ptr.size() != (int64_t)m.n_elems + 1 || m.elem_ptr[0] != 0 ||
          m.elem_ptr[m.n_elems] != (int32_t)m.elem_nodes.size())
        return "elem_ptr size";
    }
    Instance in;
    in.npe = m.npe;
    in.node_off = P.n_nodes;
    in.elem_off = P.n_elems;
    in.sub_off = P.n_sub;
    in.n_nodes = m.n_nodes;
    in.n_elems = m.n_elems;
    in.n_sub = m.n_sub;
    in.ke_off = P.ke_total;
    P.inst.push_back(in);
    P.n_nodes += m.n_nodes;
    P.n_elems += m.n_elems;
    P.n_sub += m.n_sub;
    for (int32_t e = 0; e < m.n_elems; ++e) {
      int64_t k = 3LL * npe_of(m, e);
      P.ke_total += k * k;
    }
  }
  if (P.n_nodes * 3 > INT32_MAX) return "too many DOFs for 32-bit indices";
  P.n_dofs = 3 * P.n_nodes;
  P.free_dof.assign(P.n_dofs, 1);
  P.dof_inst.assign(P.n_dofs, 0);
  P.node_glob.assign(P.n_nodes, -1);
  P.ke_off.resize(P.n_elems);
  P.elem_npe.resize(P.n_elems);
  P.elem_node_off.resize(P.n_elems);
  P.elem_nodes_flat.reserve(P.n_elems * 8);

  std::vector<std::vector<int32_t>> sub_coarse_ids(P.n_sub);  // global coarse ids per subdomain
  std::vector<std::vector<int32_t>> glob_nodes_all;           // global node ids per global glob
  std::vector<std::vector<int32_t>> glob_subs_all;            // global sub ids per glob
  std::vector<std::vector<int32_t>> glob_rdofs_all;           // near-null-space globs: free DOFs
  std::vector<std::vector<double>> glob_rows_all;             // and their rows (empty otherwise)
  std::vector<int32_t> node_deg(P.n_nodes, 0);                // |N(x)|

  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const MeshIn& m = meshes[ii];
    Instance& in = P.inst[ii];
    in.npe = m.npe;
    int64_t ko = in.ke_off;
    for (int32_t e = 0; e < m.n_elems; ++e) {
      const int64_t ge = in.elem_off + e;
      const int32_t npe = npe_of(m, e);
      P.ke_off[ge] = ko;
      ko += (int64_t)(3 * npe) * (3 * npe);
      P.elem_npe[ge] = npe;
      P.elem_node_off[ge] = (int64_t)P.elem_nodes_flat.size();
      int32_t part = m.elem_part[e];
      if (part < 0 || part >= m.n_sub) return "elem_part out of range";
      for (int32_t a = 0; a < npe; ++a) {
        int32_t nd = node_of(m, e, a);
        if (nd < 0 || nd >= m.n_nodes) return "elem_nodes out of range";
        P.elem_nodes_flat.push_back((int32_t)(in.node_off + nd));
      }
    }
    for (int32_t d : m.dirichlet) {
      if (d < 0 || d >= 3 * m.n_nodes) return "dirichlet DOF out of range";
      P.free_dof[3 * in.node_off + d] = 0;
    }
    for (int64_t d = 0; d < 3LL * m.n_nodes; ++d) P.dof_inst[3 * in.node_off + d] = ii;

    // ------------------------------------------------ N(x): subdomains per node
    std::vector<std::pair<int32_t, int32_t>> ns;
    ns.reserve(m.elem_nodes.size());
    for (int32_t e = 0; e < m.n_elems; ++e)
      for (int32_t a = 0; a < npe_of(m, e); ++a) ns.emplace_back(node_of(m, e, a), m.elem_part[e]);
    std::sort(ns.begin(), ns.end());
    ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
    std::vector<int32_t> nsp(m.n_nodes + 1, 0), nsl(ns.size());
    for (size_t k = 0; k < ns.size(); ++k) {
      nsp[ns[k].first + 1]++;
      nsl[k] = ns[k].second;
    }
    for (int32_t n = 0; n < m.n_nodes; ++n) nsp[n + 1] += nsp[n];
    std::vector<uint8_t> is_if(m.n_nodes, 0);
    for (int32_t n = 0; n < m.n_nodes; ++n) {
      int32_t deg = nsp[n + 1] - nsp[n];
      node_deg[in.node_off + n] = deg;
      bool has_free = false;
      for (int c = 0; c < 3; ++c) has_free |= P.free_dof[3 * (in.node_off + n) + c] != 0;
      is_if[n] = (deg >= 2 && has_free) ? 1 : 0;
    }
    // ------------------------------------------------ globs: key classes, connected parts
    std::map<std::vector<int32_t>, int32_t> keys;
    std::vector<int32_t> key_id(m.n_nodes, -1);
    for (int32_t n = 0; n < m.n_nodes; ++n) {
      if (!is_if[n]) continue;
      std::vector<int32_t> k(nsl.begin() + nsp[n], nsl.begin() + nsp[n + 1]);
      k.push_back(-1 - (int32_t)(m.node_tags.empty() ? 0u : m.node_tags[n]));
      auto it = keys.emplace(std::move(k), (int32_t)keys.size()).first;
      key_id[n] = it->second;
    }
    UnionFind uf(m.n_nodes);
    for (int32_t e = 0; e < m.n_elems; ++e) {
      const int32_t npe = npe_of(m, e);
      const int32_t* en = m.elem_ptr.empty() ? &m.elem_nodes[(int64_t)e * npe] : &m.elem_nodes[m.elem_ptr[e]];
      for (int32_t a = 0; a < npe; ++a) {
        int32_t ka = key_id[en[a]];
        if (ka < 0) continue;
        for (int32_t b = a + 1; b < npe; ++b)
          if (key_id[en[b]] == ka) uf.unite(en[a], en[b]);
      }
    }
    std::vector<int32_t> root_glob(m.n_nodes, -1);
    std::vector<std::vector<int32_t>> gnodes;
    for (int32_t n = 0; n < m.n_nodes; ++n) {   // ascending n: globs come out sorted by first node
      if (!is_if[n]) continue;
      int32_t r = uf.find(n);
      if (root_glob[r] < 0) {
        root_glob[r] = (int32_t)gnodes.size();
        gnodes.emplace_back();
      }
      gnodes[root_glob[r]].push_back(n);
    }
    in.glob_off = (int64_t)P.glob_kind.size();
    in.n_globs = (int32_t)gnodes.size();
    in.coarse_off = P.n_coarse;
    int32_t ncoarse = 0;
    for (size_t g = 0; g < gnodes.size(); ++g) {
      const std::vector<int32_t>& gn = gnodes[g];
      int32_t n0 = gn[0];
      int32_t deg = nsp[n0 + 1] - nsp[n0];
      int32_t nprime = deg + popcount32(m.node_tags.empty() ? 0u : m.node_tags[n0]);
      int32_t kind = (gn.size() == 1) ? kVertex : (nprime >= 3 ? kEdge : kFace);
      P.glob_kind.push_back(kind);
      P.glob_node0.push_back((int32_t)(in.node_off + n0));
      if (kind == kVertex) P.n_vertices++;
      else if (kind == kEdge) P.n_edges++;
      else P.n_faces++;
      std::vector<int32_t> gglob_nodes(gn.size());
      for (size_t k = 0; k < gn.size(); ++k) {
        gglob_nodes[k] = (int32_t)(in.node_off + gn[k]);
        P.node_glob[in.node_off + gn[k]] = (int32_t)(in.glob_off + g);
      }
      std::vector<int32_t> gsubs(nsl.begin() + nsp[n0], nsl.begin() + nsp[n0 + 1]);
      for (int32_t& s : gsubs) s += (int32_t)in.sub_off;
      std::vector<int32_t> rdofs;
      std::vector<double> rrows;
      if ((kind & primal) && nnsp && kind != kVertex) {   // rows of the glob's rigid motions
        if (m.coords.size() != 3 * (size_t)m.n_nodes) return "near-null-space primals need node coordinates";
        const int r = rigid_rows(m, gn, P.free_dof, in.node_off, rdofs, rrows);
        for (int k = 0; k < r; ++k) {
          int32_t cid = (int32_t)(in.coarse_off + ncoarse++);
          P.coarse_glob.push_back((int32_t)(in.glob_off + g));
          P.coarse_comp.push_back(k);
          for (int32_t s : gsubs) sub_coarse_ids[s].push_back(cid);
        }
      } else if (kind & primal) {
        for (int c = 0; c < 3; ++c) {
          bool any = false;
          for (int32_t nd : gglob_nodes) any |= P.free_dof[3 * (int64_t)nd + c] != 0;
          if (!any) continue;
          int32_t cid = (int32_t)(in.coarse_off + ncoarse++);
          P.coarse_glob.push_back((int32_t)(in.glob_off + g));
          P.coarse_comp.push_back(c);
          for (int32_t s : gsubs) sub_coarse_ids[s].push_back(cid);
        }
      }
      glob_rdofs_all.push_back(std::move(rdofs));
      glob_rows_all.push_back(std::move(rrows));
      glob_nodes_all.push_back(std::move(gglob_nodes));
      glob_subs_all.push_back(std::move(gsubs));
    }
    in.n_coarse = ncoarse;
    P.n_coarse += ncoarse;
  }
  for (int64_t d = 0; d < P.n_dofs; ++d) P.n_free += P.free_dof[d];

  // ---------------------------------------------------------------- subdomains
  std::vector<std::vector<int32_t>> sub_elem_lists(P.n_sub);
  for (int32_t ii = 0; ii < P.n_inst; ++ii) {
    const MeshIn& m = meshes[ii];
    for (int32_t e = 0; e < m.n_elems; ++e)
      sub_elem_lists[P.inst[ii].sub_off + m.elem_part[e]].push_back((int32_t)(P.inst[ii].elem_off + e));
  }
  std::vector<int32_t> local_of(P.n_dofs, -1);
  P.subs.resize(P.n_sub);
  P.cons_ptr.reserve(P.n_sub * 64);
  for (int64_t s = 0; s < P.n_sub; ++s) {
    SubLayout& L = P.subs[s];
    int32_t ii = 0;
    while (ii + 1 < P.n_inst && P.inst[ii + 1].sub_off <= s) ++ii;
    L.inst = ii;
    const std::vector<int32_t>& els = sub_elem_lists[s];
    if (els.empty()) return "a subdomain has no element";
    std::vector<int32_t> nodes;
    for (int32_t e : els) {
      int32_t npe = P.elem_npe[e];
      for (int32_t a = 0; a < npe; ++a) nodes.push_back(P.elem_nodes_flat[P.elem_node_off[e] + a]);
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    std::vector<int32_t> dI, dG;
    for (int32_t nd : nodes)
      for (int c = 0; c < 3; ++c) {
        int32_t d = 3 * nd + c;
        if (!P.free_dof[d]) continue;
        bool itf = node_deg[nd] >= 2;   // a node with a free DOF and |N| >= 2 is on Gamma
        (itf ? dG : dI).push_back(d);
      }
    L.nI = (int32_t)dI.size();
    L.nG = (int32_t)dG.size();
    L.dof_off = (int64_t)P.sub_dofs.size();
    for (int32_t d : dI) P.sub_dofs.push_back(d);
    for (int32_t d : dG) P.sub_dofs.push_back(d);
    for (int32_t k = 0; k < L.ni(); ++k) local_of[P.sub_dofs[L.dof_off + k]] = k;
    // element -> local DOF maps
    L.elem_off = (int64_t)P.sub_elems.size();
    L.n_elems = (int32_t)els.size();
    for (int32_t e : els) {
      P.sub_elems.push_back(e);
      P.elem_ldof_off.push_back((int64_t)P.elem_ldof.size());
      int32_t npe = P.elem_npe[e];
      for (int32_t a = 0; a < npe; ++a) {
        int32_t nd = P.elem_nodes_flat[P.elem_node_off[e] + a];
        for (int c = 0; c < 3; ++c) {
          int32_t d = 3 * nd + c;
          P.elem_ldof.push_back(P.free_dof[d] ? local_of[d] : -1);
        }
      }
    }
    // interface slots
    L.if_off = P.n_slots;
    for (int32_t d : dG) {
      P.slot_dof.push_back(d);
      P.slot_w.push_back(1.0 / (double)node_deg[d / 3]);
    }
    P.n_slots += L.nG;
    // primal constraint rows, ascending global coarse id
    const std::vector<int32_t>& cids = sub_coarse_ids[s];
    L.nc = (int32_t)cids.size();
    L.c_off = P.n_cslots;
    L.cons_off = (int64_t)P.cons_ptr.size();
    P.cons_ptr.push_back((int32_t)P.cons_idx.size());
    for (int32_t cid : cids) {
      const int32_t gg = P.coarse_glob[cid];
      if (!glob_rows_all[gg].empty()) {   // row coarse_comp of the glob's rigid-motion basis
        const std::vector<int32_t>& dd = glob_rdofs_all[gg];
        const double* row = glob_rows_all[gg].data() + (size_t)P.coarse_comp[cid] * dd.size();
        for (size_t j = 0; j < dd.size(); ++j) {
          if (row[j] == 0.0) continue;
          int32_t l = local_of[dd[j]] - L.nI;
          if (l < 0) return "internal error: constraint on an interior DOF";
          P.cons_idx.push_back(l);
          P.cons_w.push_back(row[j]);
        }
        P.cons_ptr.push_back((int32_t)P.cons_idx.size());
        P.cslot_coarse.push_back(cid);
        continue;
      }
      const std::vector<int32_t>& gn = glob_nodes_all[gg];
      int c = P.coarse_comp[cid];
      int32_t cnt = 0;
      for (int32_t nd : gn) cnt += P.free_dof[3 * (int64_t)nd + c];
      for (int32_t nd : gn) {
        int32_t d = 3 * nd + c;
        if (!P.free_dof[d]) continue;
        int32_t l = local_of[d] - L.nI;
        if (l < 0) return "internal error: constraint on an interior DOF";
        P.cons_idx.push_back(l);
        P.cons_w.push_back(1.0 / (double)cnt);
      }
      P.cons_ptr.push_back((int32_t)P.cons_idx.size());
      P.cslot_coarse.push_back(cid);
    }
    P.n_cslots += L.nc;
    for (int32_t k = 0; k < L.ni(); ++k) local_of[P.sub_dofs[L.dof_off + k]] = -1;
    P.max_local = std::max<int64_t>(P.max_local, std::max(L.ni(), L.mP()));
  }
  // ---------------------------------------------------------------- slot maps
  {
    std::vector<int32_t> ifx_of(P.n_dofs, -1);
    std::vector<int32_t> cnt;
    for (int64_t d = 0; d < P.n_dofs; ++d) {
      if (P.free_dof[d] && node_deg[d / 3] >= 2) {
        ifx_of[d] = (int32_t)P.n_ifx++;
      }
    }
    P.ifx_ptr.assign(P.n_ifx + 1, 0);
    P.slot_ifx.resize(P.n_slots);
    for (int64_t sl = 0; sl < P.n_slots; ++sl) {
      int32_t q = ifx_of[P.slot_dof[sl]];
      P.slot_ifx[sl] = q;
      P.ifx_ptr[q + 1]++;
    }
    for (int64_t q = 0; q < P.n_ifx; ++q) P.ifx_ptr[q + 1] += P.ifx_ptr[q];
    P.ifx_slots.resize(P.n_slots);
    std::vector<int32_t> fill(P.ifx_ptr.begin(), P.ifx_ptr.end() - 1);
    P.slot_owner.assign(P.n_slots, 0);
    for (int64_t sl = 0; sl < P.n_slots; ++sl) {   // slots ascend with subdomain id
      int32_t q = P.slot_ifx[sl];
      if (fill[q] == P.ifx_ptr[q]) P.slot_owner[sl] = 1;
      P.ifx_slots[fill[q]++] = (int32_t)sl;
    }
    P.coarse_ptr.assign(P.n_coarse + 1, 0);
    for (int64_t cs = 0; cs < P.n_cslots; ++cs) P.coarse_ptr[P.cslot_coarse[cs] + 1]++;
    for (int64_t k = 0; k < P.n_coarse; ++k) P.coarse_ptr[k + 1] += P.coarse_ptr[k];
    P.coarse_slots.resize(P.n_cslots);
    std::vector<int32_t> cf(P.coarse_ptr.begin(), P.coarse_ptr.end() - 1);
    for (int64_t cs = 0; cs < P.n_cslots; ++cs) P.coarse_slots[cf[P.cslot_coarse[cs]]++] = (int32_t)cs;
  }
  // ---------------------------------------------------------------- 3x3-block pattern
  {
    // node -> (element, local index)
    std::vector<int32_t> ne_ptr(P.n_nodes + 1, 0);
    for (int64_t e = 0; e < P.n_elems; ++e)
      for (int32_t a = 0; a < P.elem_npe[e]; ++a) ne_ptr[P.elem_nodes_flat[P.elem_node_off[e] + a] + 1]++;
    for (int64_t n = 0; n < P.n_nodes; ++n) ne_ptr[n + 1] += ne_ptr[n];
    std::vector<std::pair<int32_t, int32_t>> ne(ne_ptr[P.n_nodes]);
    std::vector<int32_t> f(ne_ptr.begin(), ne_ptr.end() - 1);
    for (int64_t e = 0; e < P.n_elems; ++e)
      for (int32_t a = 0; a < P.elem_npe[e]; ++a)
        ne[f[P.elem_nodes_flat[P.elem_node_off[e] + a]]++] = {(int32_t)e, a};
    P.bsr_rowptr.assign(P.n_nodes + 1, 0);
    P.bsr_cptr.push_back(0);
    struct C3 { int32_t col, e, a, b; };
    std::vector<C3> tmp;
    for (int64_t n = 0; n < P.n_nodes; ++n) {
      tmp.clear();
      for (int32_t k = ne_ptr[n]; k < ne_ptr[n + 1]; ++k) {
        int32_t e = ne[k].first, a = ne[k].second, npe = P.elem_npe[e];
        for (int32_t b = 0; b < npe; ++b) tmp.push_back({P.elem_nodes_flat[P.elem_node_off[e] + b], e, a, b});
      }
      std::sort(tmp.begin(), tmp.end(), [](const C3& x, const C3& y) {
        return x.col != y.col ? x.col < y.col : x.e < y.e;
      });
      for (size_t k = 0; k < tmp.size(); ++k) {
        if (k == 0 || tmp[k].col != tmp[k - 1].col) {
          if (k) P.bsr_cptr.push_back((int32_t)P.bsr_contrib.size());
          P.bsr_col.push_back(tmp[k].col);
          P.bsr_kstride.push_back(3 * P.elem_npe[tmp[k].e]);
        }
        int32_t nd3 = 3 * P.elem_npe[tmp[k].e];
        P.bsr_contrib.push_back(P.ke_off[tmp[k].e] + (int64_t)(3 * tmp[k].a) * nd3 + 3 * tmp[k].b);
      }
      if (!tmp.empty()) P.bsr_cptr.push_back((int32_t)P.bsr_contrib.size());
      P.bsr_rowptr[n + 1] = (int32_t)P.bsr_col.size();
    }
  }
  return "";
}

}  // namespace mbddc
