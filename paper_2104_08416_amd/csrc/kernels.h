// kernels.h -- launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

constexpr int kBlock = 256;     // threads per workgroup of the shot-batch and utility kernels
constexpr int kRowBlock = 1024; // largest workgroup of the single-shot row kernel
constexpr int kGeoShots = 1 << 16; // `geo` of the 64-shot kernel: kGeoShots + threads
constexpr int kGeoTri = 1 << 17;   // `geo` of the triangle kernel: kGeoTri + threads
constexpr int kMaxP = 7;

// Arguments of the fused step kernel. All arrays use the new (curve) numbering.
template <typename T>
struct StepArgs {
    // mesh
    // shot-batch kernel: conn [E/64][nq][64], G [E/64][3][nq][64] geometric factors
    // (11, 12, 22); row kernel: conn [E][nq], G [E][8] = six bilinear-map derivative
    // coefficients, c^2, padding
    const int32_t* conn;
    const T* G;
    const T* c2;              // [E]
    const T* dtminv;          // [N] dt / lumped mass
    int64_t E;
    int32_t S;                // shots (row length of the [N][S] state; the single-shot
                              // row kernel keeps [S][N] and is launched once per shot)
    int32_t shot;             // row kernel: the shot of this launch (sources carry shot ids)
    // byte sizes of the buffers read through bounds-checked buffer loads (each < 4 GiB)
    uint32_t conn_bytes, G_bytes, c2_bytes, state_bytes;
    // tiling
    const int32_t* tile_eb;   // [T+1] element range of each tile
    const int32_t* tile_nb;   // [T+1] owned node range of each tile
    const int32_t* tile_ns;   // [T] 64-shot kernel: owned nodes on an element edge (the first
                              //     tile_ns[t] of the range; the rest are element-interior)
    const int32_t* tile_nbd;  // [T] 64-shot atomic scatter: owned border nodes, right after
                              //     the tile_ns[t] internal ones (null otherwise)
    const int32_t* halo_b;    // [T+1]
    const int32_t* halo;      // halo elements of all tiles
    int32_t n_slices;         // S / shot_lanes
    int32_t lds_own;          // row kernel: owned-node LDS arrays hold this many entries
    // state: reads u_in, writes u_out, updates v in place
    const T* u_in;
    T* u_out;
    T* v;
    T dt;
    int32_t mode;             // 0 step, 1 r_out = K u_in, 2 r_out = dt M^-1 K u_in
    T* r_out;
    // point sources: per-tile CSR of (owned-local node, shot, weight)
    const int32_t* src_b;
    const int32_t* src_loc;
    const int32_t* src_shot;
    const T* src_w;
    double src_t, f0, t0;
    // receivers: per-tile CSR of (owned-local node, receiver index)
    const int32_t* rec_b;
    const int32_t* rec_loc;
    const int32_t* rec_idx;
    int32_t n_rec;
    T* trace;                 // record u after the step: [S][n_rec][trace_cols] (+ col)
    int64_t trace_cols, trace_col;
    const T* inj;             // inject at receivers: inj[s][r][inj_cols] (col) * inj_scale
    int64_t inj_cols, inj_col;
    T inj_scale;
    // gradient pairing: grad[e] += sum_s (Khat_e u_in_e) . (u_pair_e)
    const T* u_pair;
    double* grad;
    // global accumulator (scatter COLOUR / ATOMIC, single shot): the elements
    // [e_begin, e_begin + e_count) of the element arrays add c^2 Khat_e u_e into racc [N];
    // point lists with new node ids (src_node aligned with src_w, rec_node with rec_idx)
    T* racc;
    int32_t e_begin, e_count;
    const int32_t* src_node;
    const int32_t* rec_node;
    int32_t n_src_pts, n_rec_pts;
    // triangles: reference matrices [3][nq][nq] (Sxx, Sxy + Syx, Syy) of the nodal basis; the
    // kernel reads Sxx only (E_23 = Sxx + Syy - Sxy and E_13 = Syy are Sxx under the vertex
    // rotations of the node numbering)
    const T* tri_S;
    // 1D GLL nodes, weights and derivative matrix D[i*(p+1) + j] = l_j'(xi_i)
    T xi[kMaxP + 1];
    T w[kMaxP + 1];
    T D[(kMaxP + 1) * (kMaxP + 1)];
};

// Global-accumulator scatter (single shot, row-lane layout, elements in the order of the
// element arrays): one launch adds c^2 Khat_e u_e of the elements [e_begin, e_begin + e_count)
// into racc, with global floating-point atomics (atomic = true) or plain read-modify-write
// (atomic = false: no two elements of the range may share a node, e.g. one colour class);
// element-interior nodes take plain stores. With a.grad, also grad[e] += (Khat_e u_e).u_pair_e.
template <typename T>
hipError_t launch_elems(int p, int threads, bool atomic, const StepArgs<T>& a, hipStream_t stream);
// Node pass after the element launches, over all n nodes: r = racc, racc = 0, then
// mode 0: v -= dt M^-1 r, u_out = u_in + dt v; mode 1: r_out = r; mode 2: r_out = dt M^-1 r.
template <typename T>
hipError_t launch_node_update(const StepArgs<T>& a, int64_t n, hipStream_t stream);
// Border pass of the 64-shot atomic scatter (after the step launch, mode 0): u_out = u_in +
// dt v on the rows of the n_nodes border nodes; then traces of the n_rec receivers at border
// nodes (rec_idx, rec_node) when a.trace is set.
template <typename T>
hipError_t launch_border(const StepArgs<T>& a, const int32_t* nodes, int64_t n_nodes, const int32_t* rec_idx,
                         const int32_t* rec_node, int32_t n_rec, hipStream_t stream);
// Point terms of the global-accumulator step. phase 0 (before the element launches):
// racc -= source amplitudes at src_node (shot a.shot) and adjoint injections at rec_node;
// phase 1 (after the node pass): traces from u_out at rec_node.
template <typename T>
hipError_t launch_global_points(const StepArgs<T>& a, int phase, hipStream_t stream);

// geo = kGeoTri + threads (256/512/1024): the triangle kernel (p odd; conn [E + H][nq], records
// [E + H][4] = c_12, c_23, c_13, c^2 with K_e = c^2 (c_12 E_12 + c_23 E_23 + c_13 E_13); Sxx in
// tri_S), one shot per launch.
// geo = threads * 8 + passes (threads 256/512/1024, passes 1/2/4 batched per round of
// loads): single-shot row kernel, geometric factors computed in-kernel (shot_lanes 1);
// geo = kGeoShots + threads (256/512/1024): 64-shot kernel, one wave per element
// (shot_lanes 64, conn [E][nq], G [E][3 nq + 1] = g11, g12, g22 per node, then c^2);
// geo = 0: general shot-batch kernel.
// lds_bytes is the owned-node accumulator, the launcher adds the row kernel's stage.
// Elements per workgroup pass of the row kernel: (64 / (p+1)) * (threads / 64).
template <typename T>
hipError_t launch_step(int p, int shot_lanes, int geo, int64_t n_tiles, size_t lds_bytes,
                       const StepArgs<T>& a, hipStream_t stream);

// out[s][old] = in[new][s]  (new -> old node map)
template <typename T>
hipError_t launch_nodes_to_original(const T* in, T* out, const int32_t* node_new2old, int64_t N,
                                    int32_t S, bool shot_major, hipStream_t stream);
// out[new][s] = in[s][old]
template <typename T>
hipError_t launch_nodes_from_original(const T* in, T* out, const int32_t* node_new2old, int64_t N,
                                      int32_t S, bool shot_major, hipStream_t stream);
template <typename T>
hipError_t launch_fill(T* x, T value, int64_t n, hipStream_t stream);
template <typename T>
hipError_t launch_scale(T* x, double s, int64_t n, hipStream_t stream);
// *out += sum x^2 (out must be zeroed first)
template <typename T>
hipError_t launch_sumsq(const T* x, int64_t n, double* out, hipStream_t stream);
// out[elem_new2old[k]] = scale * acc[k]
hipError_t launch_grad_to_original(const double* acc, double* out, const int32_t* elem_new2old,
                                   int64_t E, double scale, hipStream_t stream);

// One stage of the first-order u-v system with Heun's scheme (Sec. 4.2, 4.2.1), single
// shot, tiles, halo and record layout of the single-shot kernel. V-dot = grad u at the local
// nodes of an element (Eq. v_change, F = I); R = -sum w detJ V . grad N (Eq. u_change_r_effic,
// B = -I) summed into the owned nodes; U-dot = M-bar^{-1} (R + y(src_t)) (Eq. u_change).
//   predictor (mode 0): U~ = U^n + h U-dot(V^n) into u_out; V~ is not stored.
//   fused corrector (mode 2): V~ = V^n + h grad U^n formed in registers,
//     V^{n+1} = V^n + h/2 (grad U^n + grad U~) into v_out,
//     U^{n+1} = (U^n + U~) / 2 + h/2 U-dot(V~) into u_out, and the next step's predictor
//     U~ = U^{n+1} + h U-dot(V^{n+1}) into u_pred (V^{n+1} formed for halo elements too).
// V is element-local, [E][2][nq] (element, component, local node). 512 threads, p+1 lanes
// per element.
template <typename T>
struct HeunArgs {
    const int32_t* conn;      // [E][nq]
    const T* G;               // [E][8]: bilinear-map coefficients, c^2, pad
    const T* minv_w;          // [N] 1 / M-bar (M-bar weighted by 1/c^2)
    int64_t E;
    uint32_t conn_bytes, G_bytes, state_bytes;
    const int32_t *tile_eb, *tile_nb, *halo_b, *halo;
    const T* u0;              // U^n
    const T* u1;              // U~ (corrector)
    T* u_out;
    const T* v0;              // V^n
    T* v_out;                 // V^{n+1} (corrector)
    T* u_pred;                // fused corrector: the next step's U~
    T h;
    int32_t lds_own;          // owned-node slots of the LDS prefetch arrays (64-aligned)
    const int32_t *src_b, *src_loc, *src_shot;
    const T* src_w;
    double src_t, f0, t0;
    const int32_t *rec_b, *rec_loc, *rec_idx;
    T* trace;
    int64_t trace_cols, trace_col;
    T xi[kMaxP + 1];
    T w[kMaxP + 1];
    T D[(kMaxP + 1) * (kMaxP + 1)];
};
template <typename T>
hipError_t launch_heun_stage(int p, int mode, int64_t n_tiles, size_t lds_bytes,
                             const HeunArgs<T>& a, hipStream_t stream);

// Dynamic LDS of one workgroup of the triangle kernel: the per-element stage of nq words
// (16-byte aligned), the FP64 accumulator and the three prefetch arrays.
inline size_t tri_lds_bytes(int p, int threads, int64_t lds_own, size_t word) {
    const int nq = (p + 1) * (p + 2) / 2, nqp = (nq + 3) & ~3, epb = (64 / nq) * (threads / 64);
    return (size_t)epb * nqp * word + (size_t)lds_own * 8 + (size_t)3 * lds_own * word;
}
// Dynamic LDS of one workgroup of the single-shot row kernel: the per-element stage
// (16-byte aligned rows of nq words), the FP64 accumulator and the three prefetch arrays
// (v, u, dt/M) of lds_own entries each.
inline size_t rows_lds_bytes(int p, int threads, int64_t lds_own, size_t word) {
    const int n = p + 1, nqp = (n * n + 3) & ~3, epb = (64 / n) * (threads / 64);
    return (size_t)epb * nqp * word + (size_t)lds_own * 8 + (size_t)3 * lds_own * word;
}
// Heun stages (512 threads): stage, one FP64 accumulator (two for the fused corrector,
// mode 2) and, in FP32 only, three prefetch arrays of lds_own entries.
inline size_t heun_lds_bytes(int p, int mode, int64_t lds_own, size_t word) {
    const int n = p + 1, nqp = (n * n + 3) & ~3, epb = (64 / n) * (kRowBlock / 2 / 64);
    return (size_t)epb * nqp * word + (size_t)(mode == 2 ? 2 : 1) * lds_own * 8 +
           (word == 4 ? (size_t)3 * lds_own * word : 0);
}
constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

}  // namespace sem
