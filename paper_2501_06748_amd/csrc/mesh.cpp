// Mesh topology for scaled-boundary polygons (host side, once per mesh).
//
// Geometry follows the scaling-centre transformation of the paper (Section
// "Scaled boundary discretization"): every point of an element is the centre
// plus xi times a point of the boundary, and the boundary is interpolated by
// straight segments between consecutive loop nodes.  The scaling centre must
// see every segment counter-clockwise (det J_b > 0), which is checked here.
//
// The coarse nodal system couples the boundary nodes of each element
// (S_e u_n = f_hat); this file builds the node -> (element, slot) map used to
// gather element sources without atomics, and the CSR pattern of
// K_g = sum_e L_e^T S_e L_e together with, for every CSR entry, the list of
// element-matrix entries that sum into it (a deterministic assembly).

#include <algorithm>
#include <cmath>
#include <map>

#include "sbfwi_internal.h"

static int upload_mesh(sbfwi_mesh_s* m, const std::vector<int64_t>& loop_nodes,
                       const std::vector<double>& loop_xy, const std::vector<double>& centre,
                       const std::vector<int64_t>& node_ptr, const std::vector<int64_t>& node_slot,
                       const std::vector<int32_t>& col, const std::vector<int64_t>& diag,
                       const std::vector<int64_t>& tr, const std::vector<int64_t>& cptr,
                       const std::vector<int64_t>& csrc) {
  SBFWI_CHECK(sbfwi_upload(&m->d.nb, m->h_nb));
  SBFWI_CHECK(sbfwi_upload(&m->d.nr, m->h_nr));
  SBFWI_CHECK(sbfwi_upload(&m->d.loop_off, m->h_loop_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.par_off, m->h_par_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.int_off, m->h_int_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.x_off, m->h_x_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.finv_off, m->h_finv_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.dense_off, m->h_dense_off));
  SBFWI_CHECK(sbfwi_upload(&m->d.loop_nodes, loop_nodes));
  SBFWI_CHECK(sbfwi_upload(&m->d.loop_xy, loop_xy));
  SBFWI_CHECK(sbfwi_upload(&m->d.centre, centre));
  SBFWI_CHECK(sbfwi_upload(&m->d.node_ptr, node_ptr));
  SBFWI_CHECK(sbfwi_upload(&m->d.node_slot, node_slot));
  SBFWI_CHECK(sbfwi_upload(&m->d.row_ptr, m->h_row_ptr));
  SBFWI_CHECK(sbfwi_upload(&m->d.col, col));
  SBFWI_CHECK(sbfwi_upload(&m->d.diag_idx, diag));
  SBFWI_CHECK(sbfwi_upload(&m->d.tr_idx, tr));
  SBFWI_CHECK(sbfwi_upload(&m->d.contrib_ptr, cptr));
  SBFWI_CHECK(sbfwi_upload(&m->d.contrib_src, csrc));
  for (int c = 0; c < 3; ++c) SBFWI_CHECK(sbfwi_upload(&m->class_elems[c], m->h_class_elems[c]));
  SBFWI_CHECK(sbfwi_upload(&m->d.elem_by_cost, m->h_elem_by_cost));
  // sliced ELL layout of the coarse pattern: slices of ELL_SLICE rows, each
  // padded to its widest row rounded up to ELL_LPR entries; chunk c of a slice
  // stores entries k = c*ELL_LPR .. c*ELL_LPR + ELL_LPR-1 of every row, row-major
  // inside the chunk: position = off + (c * ELL_SLICE + row_in_slice) * ELL_LPR + k % ELL_LPR
  const int64_t n = m->n_nodes, ns = (n + ELL_SLICE - 1) / ELL_SLICE;
  std::vector<int64_t> eoff(ns + 1, 0);
  std::vector<int32_t> ew(ns, 0);
  for (int64_t sl = 0; sl < ns; ++sl) {
    int64_t w = 0;
    for (int64_t r = sl * ELL_SLICE; r < std::min(n, (sl + 1) * ELL_SLICE); ++r)
      w = std::max(w, m->h_row_ptr[r + 1] - m->h_row_ptr[r]);
    const int64_t chunks = (w + ELL_LPR - 1) / ELL_LPR;
    ew[sl] = (int32_t)chunks;
    eoff[sl + 1] = eoff[sl] + chunks * ELL_SLICE * ELL_LPR;
  }
  std::vector<int32_t> ecol(eoff[ns]);
  std::vector<int64_t> epos(m->nnz);
  for (int64_t sl = 0; sl < ns; ++sl)
    for (int64_t lr = 0; lr < ELL_SLICE; ++lr) {
      int64_t r = sl * ELL_SLICE + lr;
      for (int64_t k = 0; k < (int64_t)ew[sl] * ELL_LPR; ++k) {
        int64_t pos = eoff[sl] + ((k / ELL_LPR) * ELL_SLICE + lr) * ELL_LPR + k % ELL_LPR;
        int64_t q = r < n ? m->h_row_ptr[r] + k : -1;
        if (r < n && q < m->h_row_ptr[r + 1]) {
          ecol[pos] = (int32_t)m->h_col64[q];
          epos[q] = pos;
        } else {
          ecol[pos] = (int32_t)(r < n ? r : 0);
        }
      }
    }
  m->d.n_ell = eoff[ns];
  SBFWI_CHECK(sbfwi_upload(&m->d.ell_off, eoff));
  SBFWI_CHECK(sbfwi_upload(&m->d.ell_w, ew));
  SBFWI_CHECK(sbfwi_upload(&m->d.ell_col, ecol));
  SBFWI_CHECK(sbfwi_upload(&m->d.ell_pos, epos));
  return SBFWI_OK;
}

void sbfwi_mesh_free(sbfwi_mesh_s* m) {
  if (!m) return;
  MeshDev& d = m->d;
  void* ptrs[] = {d.nb, d.nr, d.loop_off, d.par_off, d.int_off, d.x_off, d.finv_off,
                  d.dense_off, d.loop_nodes, d.loop_xy, d.centre, d.node_ptr, d.node_slot,
                  d.row_ptr, d.col, d.diag_idx, d.tr_idx, d.contrib_ptr, d.contrib_src,
                  d.ell_off, d.ell_w, d.ell_col, d.ell_pos, d.elem_by_cost,
                  m->class_elems[0], m->class_elems[1], m->class_elems[2]};
  for (void* p : ptrs) sbfwi_dev_free(p);
  sbfwi_direct_sym_free(m->dsym);
  delete m;
}

extern "C" int sbfwi_build_mesh(const double* node_xy, int64_t n_nodes, const int64_t* elem_ptr,
                                const int64_t* elem_nodes, int64_t n_elem,
                                const double* centre_xy, const int32_t* n_r, double xi0,
                                sbfwi_mesh* out) {
  if (!out) return sbfwi_fail(SBFWI_EINVAL, "out is NULL");
  *out = nullptr;
  if (!node_xy || !elem_ptr || !elem_nodes || !n_r || n_nodes <= 0 || n_elem <= 0)
    return sbfwi_fail(SBFWI_EINVAL, "empty or NULL mesh arrays");
  if (n_nodes >= (int64_t)INT32_MAX) return sbfwi_fail(SBFWI_EINVAL, "too many nodes");
  if (!(xi0 > 0.0 && xi0 < 0.5)) return sbfwi_fail(SBFWI_EINVAL, "xi0 must be in (0, 0.5)");
  if (elem_ptr[0] != 0) return sbfwi_fail(SBFWI_EINVAL, "elem_ptr[0] must be 0");
  sbfwi_mesh_s* m = new sbfwi_mesh_s();
  m->n_nodes = n_nodes;
  m->n_elem = n_elem;
  m->xi0 = xi0;
  m->h_nb.resize(n_elem);
  m->h_nr.resize(n_elem);
  std::vector<double> centre(2 * n_elem);
  for (int64_t e = 0; e < n_elem; ++e) {
    int64_t nb = elem_ptr[e + 1] - elem_ptr[e];
    if (nb < 3 || nb > SBFWI_MAX_NB) {
      sbfwi_mesh_free(m);
      return sbfwi_fail(SBFWI_EINVAL, "element %lld has %lld boundary nodes (3..%d allowed)",
                        (long long)e, (long long)nb, SBFWI_MAX_NB);
    }
    if (n_r[e] < 3 || n_r[e] > 128) {
      sbfwi_mesh_free(m);
      return sbfwi_fail(SBFWI_EINVAL, "element %lld has N_r = %d (3..128 allowed)", (long long)e, n_r[e]);
    }
    m->h_nb[e] = (int32_t)nb;
    m->h_nr[e] = n_r[e];
    double cx, cy;
    if (centre_xy) {
      cx = centre_xy[2 * e];
      cy = centre_xy[2 * e + 1];
    } else {  // area centroid of the polygon
      double a2 = 0, sx = 0, sy = 0;
      for (int64_t i = 0; i < nb; ++i) {
        int64_t p = elem_nodes[elem_ptr[e] + i], q = elem_nodes[elem_ptr[e] + (i + 1) % nb];
        if (p < 0 || p >= n_nodes || q < 0 || q >= n_nodes) {
          sbfwi_mesh_free(m);
          return sbfwi_fail(SBFWI_EINVAL, "element %lld references a node out of range", (long long)e);
        }
        double x0 = node_xy[2 * p], y0 = node_xy[2 * p + 1], x1 = node_xy[2 * q], y1 = node_xy[2 * q + 1];
        double cr = x0 * y1 - x1 * y0;
        a2 += cr;
        sx += (x0 + x1) * cr;
        sy += (y0 + y1) * cr;
      }
      if (!(a2 > 0)) {
        sbfwi_mesh_free(m);
        return sbfwi_fail(SBFWI_EINVAL, "element %lld is not counter-clockwise", (long long)e);
      }
      cx = sx / (3.0 * a2);
      cy = sy / (3.0 * a2);
    }
    centre[2 * e] = cx;
    centre[2 * e + 1] = cy;
    for (int64_t i = 0; i < nb; ++i) {  // det J_b > 0 on every segment
      int64_t p = elem_nodes[elem_ptr[e] + i], q = elem_nodes[elem_ptr[e] + (i + 1) % nb];
      if (p < 0 || p >= n_nodes || q < 0 || q >= n_nodes) {
        sbfwi_mesh_free(m);
        return sbfwi_fail(SBFWI_EINVAL, "element %lld references a node out of range", (long long)e);
      }
      double ax = node_xy[2 * p] - cx, ay = node_xy[2 * p + 1] - cy;
      double bx = node_xy[2 * q] - cx, by = node_xy[2 * q + 1] - cy;
      double area2 = ax * by - ay * bx;
      double scale = (ax * ax + ay * ay + bx * bx + by * by);
      if (!(area2 > 1e-12 * scale)) {
        sbfwi_mesh_free(m);
        return sbfwi_fail(SBFWI_EINVAL,
                          "element %lld segment %lld: det J_b <= 0 (loop not CCW or not star-convex "
                          "with respect to its scaling centre)", (long long)e, (long long)i);
      }
    }
  }
  // offsets
  auto prefix = [&](std::vector<int64_t>& off, auto size_of) {
    off.assign(n_elem + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e) off[e + 1] = off[e] + size_of(e);
  };
  prefix(m->h_loop_off, [&](int64_t e) { return (int64_t)m->h_nb[e]; });
  prefix(m->h_par_off, [&](int64_t e) { return (int64_t)m->h_nb[e] * m->h_nr[e]; });
  prefix(m->h_int_off, [&](int64_t e) { return (int64_t)m->h_nb[e] * (m->h_nr[e] - 1); });
  prefix(m->h_x_off, [&](int64_t e) { return (int64_t)m->h_nb[e] * (m->h_nr[e] + 2); });
  prefix(m->h_finv_off, [&](int64_t e) { return (int64_t)m->h_nb[e] * m->h_nb[e] * (m->h_nr[e] - 1); });
  prefix(m->h_dense_off, [&](int64_t e) { return (int64_t)m->h_nb[e] * m->h_nb[e]; });
  m->n_loop = m->h_loop_off[n_elem];
  m->n_params = m->h_par_off[n_elem];
  m->n_int = m->h_int_off[n_elem];
  m->n_x = m->h_x_off[n_elem];
  m->n_finv = m->h_finv_off[n_elem];
  m->n_dense = m->h_dense_off[n_elem];
  std::vector<int64_t> loop_nodes(elem_nodes, elem_nodes + m->n_loop);
  std::vector<double> loop_xy(2 * m->n_loop);
  for (int64_t q = 0; q < m->n_loop; ++q) {
    loop_xy[2 * q] = node_xy[2 * loop_nodes[q]];
    loop_xy[2 * q + 1] = node_xy[2 * loop_nodes[q] + 1];
  }
  for (int64_t e = 0; e < n_elem; ++e) {  // a node may appear once per loop
    std::vector<int64_t> ids(loop_nodes.begin() + m->h_loop_off[e], loop_nodes.begin() + m->h_loop_off[e + 1]);
    std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end()) {
      sbfwi_mesh_free(m);
      return sbfwi_fail(SBFWI_EINVAL, "element %lld repeats a node in its loop", (long long)e);
    }
  }
  // node -> loop slots
  std::vector<int64_t> node_ptr(n_nodes + 1, 0), node_slot(m->n_loop);
  for (int64_t q = 0; q < m->n_loop; ++q) node_ptr[loop_nodes[q] + 1]++;
  for (int64_t n = 0; n < n_nodes; ++n) node_ptr[n + 1] += node_ptr[n];
  {
    std::vector<int64_t> fill(node_ptr.begin(), node_ptr.end() - 1);
    for (int64_t q = 0; q < m->n_loop; ++q) node_slot[fill[loop_nodes[q]]++] = q;
  }
  // coarse pattern: union of element node pairs, sorted columns per row
  std::vector<std::vector<int64_t>> rows(n_nodes);
  for (int64_t e = 0; e < n_elem; ++e) {
    int64_t o = m->h_loop_off[e], nb = m->h_nb[e];
    for (int64_t i = 0; i < nb; ++i)
      for (int64_t j = 0; j < nb; ++j) rows[loop_nodes[o + i]].push_back(loop_nodes[o + j]);
  }
  m->h_row_ptr.assign(n_nodes + 1, 0);
  for (int64_t r = 0; r < n_nodes; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    m->h_row_ptr[r + 1] = m->h_row_ptr[r] + (int64_t)v.size();
  }
  m->nnz = m->h_row_ptr[n_nodes];
  std::vector<int32_t> col(m->nnz);
  m->h_col64.resize(m->nnz);
  std::vector<int64_t> diag(n_nodes, -1);
  for (int64_t r = 0; r < n_nodes; ++r) {
    for (size_t t = 0; t < rows[r].size(); ++t) {
      int64_t q = m->h_row_ptr[r] + (int64_t)t;
      col[q] = (int32_t)rows[r][t];
      m->h_col64[q] = rows[r][t];
      if (rows[r][t] == r) diag[r] = q;
    }
  }
  for (int64_t r = 0; r < n_nodes; ++r) {
    if (diag[r] < 0) {
      sbfwi_mesh_free(m);
      return sbfwi_fail(SBFWI_EINVAL, "node %lld belongs to no element", (long long)r);
    }
  }
  auto find = [&](int64_t r, int64_t c) {
    auto b = m->h_col64.begin() + m->h_row_ptr[r], en = m->h_col64.begin() + m->h_row_ptr[r + 1];
    return (int64_t)(std::lower_bound(b, en, c) - m->h_col64.begin());
  };
  std::vector<int64_t> tr(m->nnz);
  for (int64_t r = 0; r < n_nodes; ++r)
    for (int64_t q = m->h_row_ptr[r]; q < m->h_row_ptr[r + 1]; ++q) tr[q] = find(m->h_col64[q], r);
  // assembly lists, in element order for every entry
  std::vector<int64_t> cnt(m->nnz + 1, 0);
  std::vector<int64_t> entry_of;  // per (e, i, j) its CSR position
  entry_of.reserve(m->n_dense);
  for (int64_t e = 0; e < n_elem; ++e) {
    int64_t o = m->h_loop_off[e], nb = m->h_nb[e];
    for (int64_t i = 0; i < nb; ++i)
      for (int64_t j = 0; j < nb; ++j) {
        int64_t q = find(loop_nodes[o + i], loop_nodes[o + j]);
        entry_of.push_back(q);
        cnt[q + 1]++;
      }
  }
  for (int64_t q = 0; q < m->nnz; ++q) cnt[q + 1] += cnt[q];
  std::vector<int64_t> csrc(m->n_dense);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < m->n_dense; ++t) csrc[fill[entry_of[t]]++] = t;
  }
  m->n_contrib = m->n_dense;
  // elements by decreasing sweep cost N_r n_b^2 (ties by index): the blocks of
  // a launch are dispatched roughly in index order, so long sweeps start first
  std::vector<int32_t> by_cost(n_elem);
  for (int64_t e = 0; e < n_elem; ++e) by_cost[e] = (int32_t)e;
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int32_t x, int32_t y) {
    return (int64_t)m->h_nr[x] * m->h_nb[x] * m->h_nb[x] > (int64_t)m->h_nr[y] * m->h_nb[y] * m->h_nb[y];
  });
  for (int32_t e : by_cost) {
    int c = m->h_nb[e] <= 8 ? 0 : (m->h_nb[e] <= 16 ? 1 : 2);
    m->h_class_elems[c].push_back(e);
    m->class_nmax[c] = std::max(m->class_nmax[c], m->h_nr[e] - 1);
  }
  m->h_elem_by_cost = by_cost;
  m->d.n_nodes = n_nodes;
  m->d.n_elem = n_elem;
  m->d.n_loop = m->n_loop;
  m->d.nnz = m->nnz;
  m->d.xi0 = xi0;
  int rc = upload_mesh(m, loop_nodes, loop_xy, centre, node_ptr, node_slot, col, diag, tr, cnt, csrc);
  if (rc == SBFWI_OK) rc = sbfwi_direct_symbolic(m, node_xy);
  if (rc != SBFWI_OK) {
    sbfwi_mesh_free(m);
    return rc;
  }
  *out = m;
  return SBFWI_OK;
}

extern "C" int sbfwi_mesh_info(sbfwi_mesh m, int64_t* out) {
  if (!m || !out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  out[0] = m->n_nodes;
  out[1] = m->n_elem;
  out[2] = m->n_params;
  out[3] = m->nnz;
  out[4] = m->n_int;
  return SBFWI_OK;
}

extern "C" int sbfwi_coarse_pattern(sbfwi_mesh m, int64_t* row_ptr, int64_t* col) {
  if (!m || !row_ptr || !col) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  std::copy(m->h_row_ptr.begin(), m->h_row_ptr.end(), row_ptr);
  std::copy(m->h_col64.begin(), m->h_col64.end(), col);
  return SBFWI_OK;
}

extern "C" void sbfwi_destroy_mesh(sbfwi_mesh m) { sbfwi_mesh_free(m); }
