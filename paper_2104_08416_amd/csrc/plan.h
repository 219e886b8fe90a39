// plan.h -- host-side setup of the Hilbert-ordered SEM step (internal to the library).
//
// The plan holds everything the device step needs, in the NEW (curve) numbering:
// element-major structure-of-arrays connectivity and geometric factors, the lumped
// mass, the workgroup tiling with each tile's owned node range and halo elements, and
// the permutations back to the original numbering.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sem {

struct MeshIn {
    int64_t nv = 0, ne = 0;
    const double* vxy = nullptr;
    const int32_t* quad = nullptr;    // [ne][nvpe] CCW vertex ids
    const double* c2 = nullptr;
    int nvpe = 4;                     // vertices per element: 4 quadrilaterals, 3 triangles
};

struct PlanOptions {
    int p = 4;
    int elem_order = 0;      // 0 hilbert, 1 morton, 2 lex, 3 random
    int node_order = 0;      // 0 first touch + degree, 1 original
    uint64_t seed = 3;
    double dt = 0.0;
    double cfl = 0.3;
    int tile_elems = 0;      // > 0: fixed tiles of this many elements
    int tile_items = 256;    // adaptive tiles: own + halo elements per tile at most this
    int max_owned = 1 << 30; // adaptive tiles: owned nodes per tile at most this
    // Regroup each tile's owned nodes: nodes of two or more elements first, then nodes of
    // a single element (kept in registers by the 64-shot kernel); max_owned then bounds
    // the first group only.
    bool split_single = false;
    // with split_single: border mode (see split_border)
    bool border = false;
};

struct Plan {
    int p = 0, n = 0, nq = 0;
    int nvpe = 4;                            // 4 quadrilaterals (GLL tensor), 3 triangles
    int64_t ne = 0, nn = 0, nv = 0;
    double dt = 0.0;
    // 1D GLL ingredients
    std::vector<double> xi, w, D;            // D[i*n + j] = l_j'(xi_i)
    // original numbering
    std::vector<int32_t> conn0;              // [ne][nq] original node ids
    std::vector<double> node_xy;             // [nn][2] original numbering
    // permutations
    std::vector<int32_t> elem_new2old, elem_old2new;
    std::vector<int32_t> node_new2old, node_old2new;
    // device-bound arrays, new numbering
    std::vector<int32_t> conn_soa;           // [nq][ne] new node ids
    std::vector<double> G_soa;               // [3][nq][ne] w_a w_b detJ J^-1 J^-T (11, 12, 22)
    std::vector<double> bilin;               // [6][ne] x_xi = c0 + c2 eta, x_eta = c1 + c2 xi,
                                             //         y_xi = c3 + c5 eta, y_eta = c4 + c5 xi
    std::vector<double> c2;                  // [ne]
    std::vector<double> minv;                // [nn] 1 / lumped mass
    // tiling (new numbering): tile t has elements [tile_eb[t], tile_eb[t+1]), owns nodes
    // [tile_nb[t], tile_nb[t+1]), and recomputes halo[halo_b[t] .. halo_b[t+1]).
    int tile_elems = 0;                      // fixed tile size, 0 when adaptive
    int tile_items = 0;                      // adaptive cap on own + halo elements
    std::vector<int32_t> tile_eb, tile_nb, halo_b, halo;
    int32_t max_owned = 0;
    // split_single: tile t's owned nodes [tile_nb[t], tile_nb[t] + tile_ns[t]) lie on an
    // element edge (nodes of two or more elements, or on the domain boundary); the rest of its
    // range are element-interior nodes of its own elements.
    std::vector<int32_t> tile_ns;
    int32_t max_shared = 0;
    // border mode (64 shot lanes with global atomics): tile t's owned range is
    // [internal edge: tile_ns[t] | border: tile_nbd[t] | element-interior]; a border node is
    // touched by elements of two or more tiles; border_nodes lists them all (tile by tile)
    std::vector<int32_t> tile_nbd, border_nodes;
    // greedy element colouring in the new element order (Sec. 5): colour[k] of new
    // element k; two elements sharing a global node never share a colour
    std::vector<int32_t> colour;
    int32_t n_colours = 0;
    double reorder_seconds = 0.0;
    // triangles: reference nodes [nq][2], weights [nq], reference matrices [3][nq][nq]
    // (Sxx, Sxy + Syx, Syy) and per-element factors det J J^-1 J^-T [3][ne] (g11, g12, g22,
    // new order); dt_from_stability: dt is set to a fraction of the stability limit once
    // the device power iteration has estimated it
    std::vector<double> tri_xy, tri_w, tri_S, tri_G;
    bool dt_from_stability = false;
};

// Triangles (tri.cpp): local node count, local index of node (i, j), the reference nodes,
// weights and stiffness matrices, and the original global numbering.
int tri_nq(int p);
int tri_lidx(int i, int j, int p);
std::string tri_reference(int p, const std::vector<double>& gll_x, std::vector<double>& xy,
                          std::vector<double>& w, std::vector<double>& S);
// Checks the vertex symmetry the triangle kernel relies on: E_23 = Sxx + Syy - Sxy and
// E_13 = Syy are Sxx with rows and columns permuted by the vertex rotations (i, j, k) ->
// (j, k, i) and (k, i, j) of the local node numbering.
std::string tri_symmetry(int p, const std::vector<double>& S);
std::string tri_number_nodes(const MeshIn& mesh, int p, std::vector<int32_t>& conn, int64_t& nn);

// Fills `plan` or returns a non-empty error string; `code` receives the sem_status.
std::string build_plan(const MeshIn& mesh, const PlanOptions& opt, Plan& plan, int& code);

// (Re)build the tiling: fixed tiles of `tile_elems` elements when > 0, else adaptive tiles
// that grow along the element order while own + halo elements <= tile_items and owned
// nodes (with split_single: owned nodes on an element edge) <= max_owned.
// split_single then regroups every tile's owned range and renumbers the nodes.
void build_tiles(Plan& plan, int tile_elems, int tile_items, int max_owned, bool split_single);

// Border mode on top of build_tiles(..., split_single = true): split every tile's edge
// nodes into those whose elements all lie in the tile (first) and border nodes (touched
// by another tile's elements), renumber the nodes, fill tile_ns / tile_nbd / border_nodes
// and drop the halo lists (tiles then process their own elements only).
void split_border(Plan& plan);

// Cell index along the generalized Hilbert curve over a W x H grid.
int64_t hilbert_index(int64_t W, int64_t H, int64_t cx, int64_t cy);

// First-fit colouring of the elements in the plan's element order: each element takes the
// smallest colour not used by an earlier element that shares a global node with it.
// Returns false when more than 64 colours would be needed.
bool colour_elements(Plan& plan);

// Nearest global node (original numbering) of each of n points xy[2n]; equal distances go
// to the lowest id (the same node as a scan of all nodes). The nodes are bucketed on a grid
// once per call, so a call costs O(nn + n * nodes near each point).
void nearest_nodes(const Plan& plan, int64_t n, const double* xy, int32_t* out);

// Geometric factors of one element (original numbering) at its (p+1)^2 GLL points.
void element_geometry(const Plan& plan, const MeshIn& mesh, int64_t e, double* g11, double* g12,
                      double* g22, double* det);

}  // namespace sem
