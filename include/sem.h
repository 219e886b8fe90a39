/*
 * sem.h -- C ABI of the Hilbert-ordered spectral-element wave propagator for MI355X (gfx950).
 *
 * The library advances the 2D acoustic wave equation u_tt = div(c^2 grad u) + s on a
 * conforming quadrilateral mesh with Gauss-Lobatto-Legendre (GLL) nodes of order p,
 * with explicit leapfrog steps. Elements are relabelled along a space-filling curve and
 * global nodes are relabelled by first touch in that element order, with each element's
 * new nodes sorted by ascending degree (Araujo, Gross, Xavier-de-Souza 2021, Sec. 4.3).
 * One time step gathers each element's nodal values, applies the tensor-product stiffness
 * (derivative matrix D, geometric factors, D^T; Sec. 4.2, Eqs. deriv_u and R),
 * scatter-adds into the global vector and applies the diagonal-mass-inverse update
 * (Eq. u_change, with the point sources of Alg. 3).
 *
 * Conventions shared by every call
 *   - All user-visible arrays use the ORIGINAL numbering: elements in input order; global
 *     nodes numbered vertices first (node id = vertex id), then the p-1 interior nodes of
 *     each edge in order of first appearance over (element, local edge 0..3) counted from
 *     the edge's lower-id vertex, then the (p-1)^2 interior nodes of each element. The
 *     internal relabelling never leaks through the ABI except via sem_get_permutations.
 *   - Local edge k of a quad runs from corner k to corner (k+1)%4; corners are CCW.
 *   - Return value of every int-returning call: SEM_OK (0) or a negative SEM_ERR_* code;
 *     sem_last_error() then describes the failure. No C++ exception crosses the ABI.
 *   - Host pointers (const double*, const int32_t* in sem_mesh, xy arrays, permutation
 *     outputs) are read or written synchronously; the library copies inputs, the caller
 *     keeps ownership. Device pointers (names ending in _dev) are borrowed for
 *     stream-ordered use on the context's stream and must stay valid until that stream
 *     has executed the call's work.
 *   - A context is not thread-safe; calls on one context must be serialised.
 */
#ifndef SEM_H_
#define SEM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx sem_ctx;

enum sem_status {
    SEM_OK = 0,
    SEM_ERR_INVALID_ARG = -1,  /* null pointer, out-of-range id or option, bad size   */
    SEM_ERR_BAD_MESH = -2,     /* non-positive Jacobian, non-conforming or CW element */
    SEM_ERR_UNSTABLE_DT = -3,  /* dt >= 2/sqrt(lambda_max(M^-1 K)) (power iteration) */
    SEM_ERR_HIP = -4,          /* a HIP runtime call failed                           */
    SEM_ERR_OOM = -5,          /* device or host allocation failed                    */
    SEM_ERR_NO_DEVICE = -6     /* compute call on a host-only context                 */
};

enum sem_precision { SEM_F32 = 0, SEM_F64 = 1 };
/* Element orders: the generalized Hilbert curve (Sec. 4.3), Morton, lexicographic (input),
 * random (splitmix64 of seed ^ id), and the benchmark section's node-walk strategies
 * (Sec. 5): Node Connectivity and Node Distance, breadth-first walks over the mesh
 * vertices keyed on vertex degree or on the distance to the lower-left corner, each
 * visited vertex listing its not-yet-listed elements in ascending id. */
enum sem_elem_order { SEM_ORDER_HILBERT = 0, SEM_ORDER_MORTON = 1, SEM_ORDER_LEX = 2,
                      SEM_ORDER_RANDOM = 3, SEM_ORDER_CONNECTIVITY = 4, SEM_ORDER_DISTANCE = 5 };
enum sem_node_order { SEM_NODES_FIRST_TOUCH = 0, SEM_NODES_ORIGINAL = 1 };
enum sem_field { SEM_FIELD_U = 0, SEM_FIELD_V = 1 };
/* SEM_FORM_LEAPFROG: u_tt = div(c^2 grad u) + s, unweighted lumped mass, leapfrog.
 * SEM_FORM_HEUN: the paper's first-order system (Sec. 4.1-4.2.1) with rho = 1, K = c^2:
 * (1/c^2) u_t = div v + s, v_t = grad u, v stored per element at its GLL nodes, lumped
 * mass weighted by 1/c^2, Heun predictor-corrector (two operator evaluations per step).
 * Single shot only; sources enter as y(t) in the u equation; no adjoint; SEM_FIELD_V is
 * not available (v is element-local). Each step's launch also computes the next step's
 * predictor, kept in the context; sem_reset, sem_set_field and sem_set_sources drop it,
 * so the next step recomputes it. */
enum sem_formulation { SEM_FORM_LEAPFROG = 0, SEM_FORM_HEUN = 1 };
/* How a step sums the element contributions r_e into the shared global nodes (the race of
 * the accumulation in Alg. 2; Sec. 5 resolves it by element colouring):
 *   SEM_SCATTER_LDS_ATOMIC: each workgroup owns a contiguous range of nodes, sums every
 *     contribution to them in LDS (FP64 LDS atomics) and recomputes the neighbouring
 *     elements of other workgroups that touch them; one launch per step, no global r.
 *   SEM_SCATTER_COLOUR: the paper's scheme. Elements are greedily coloured in the element
 *     order (two elements sharing a node differ in colour), one launch per colour adds
 *     r_e into a global r with plain read-modify-write (no two elements of a colour share
 *     a node), then one launch applies the update and clears r.
 *   SEM_SCATTER_ATOMIC: single shot: one launch over all elements adds r_e into a global r
 *     with global floating-point atomics, then the update launch. Batches of 64-shot lanes:
 *     tiles process their own elements only (no halo); nodes whose elements all lie in the
 *     tile are summed in LDS, border nodes take -dt/M r_e on their 64-shot rows of v with
 *     global atomics, and a border pass after the step forms their u.
 *   SEM_SCATTER_AUTO: the fastest measured on MI355X for the context's kernel, which is
 *     LDS_ATOMIC for every configuration measured so far.
 * COLOUR is built for the single-shot leapfrog step on quadrilaterals, ATOMIC for that step
 * and for batches of 64-shot lanes. */
enum sem_scatter { SEM_SCATTER_AUTO = 0, SEM_SCATTER_LDS_ATOMIC = 1, SEM_SCATTER_COLOUR = 2,
                   SEM_SCATTER_ATOMIC = 3 };

/* Input mesh (host arrays, original numbering). */
typedef struct {
    int64_t n_vertices;
    const double* vxy;       /* [n_vertices][2] vertex coordinates                    */
    int64_t n_elements;
    const int32_t* quad;     /* [n_elements][vertices_per_element] CCW vertex ids      */
    const double* c2;        /* [n_elements] squared wave speed, > 0                   */
    int32_t vertices_per_element;
                             /* 4 (or 0): quadrilaterals, GLL tensor nodes of order p.  *
                              * 3: the paper's element (Sec. 4.2): affine triangles     *
                              * with the (p+1)(p+2)/2 Blyth-Pozrikidis nodes (GLL nodes *
                              * on every edge) and the nodal basis dual to them, the    *
                              * nodes doubling as quadrature points (weights = integrals *
                              * of the basis functions). Odd p only (the weights are not *
                              * all positive at even p); leapfrog, LDS scatter; one     *
                              * launch per shot; default dt = 0.6 times the estimated   *
                              * stability limit 2 / sqrt(lambda_max). Local node (i, j) *
                              * at x = (1 + 2 v_i - v_j - v_k) / 3, y likewise, k =     *
                              * p - i - j, v the GLL nodes on [0, 1]; original numbering *
                              * as for quadrilaterals (vertices, edge nodes by first    *
                              * appearance over local edges 0..2, interior nodes).     */
} sem_mesh;

/* Options of sem_create. Zero-initialise, then set what is needed. */
typedef struct {
    int32_t p;               /* GLL order, 1..7                                         */
    int32_t precision;       /* sem_precision                                           */
    int32_t elem_order;      /* sem_elem_order                                          */
    int32_t node_order;      /* sem_node_order; device contexts need FIRST_TOUCH        */
    uint64_t seed;           /* seed of SEM_ORDER_RANDOM                                */
    int32_t n_shots;         /* independent wavefields advanced together, >= 1          */
    int32_t device;          /* HIP device ordinal; -1 = host-only (setup, no compute)  */
    double dt;               /* time step; 0 = cfl * min_e(dx_min,e / c_e)              */
    double cfl;              /* CFL number of the default dt; 0 = 0.3                  */
    void* stream;            /* hipStream_t for all device work; NULL = default stream */
    int32_t tile_elems;      /* > 0: fixed tiles of this many elements; 0 = adaptive     */
    int32_t shot_lanes;      /* shots per element inside a workgroup; 0 = automatic     *
                              * (64 when n_shots % 64 == 0: one wave per element, one    *
                              * shot per lane)                                          */
    int32_t tile_items;      /* adaptive tiles: own + halo elements per tile; 0 = auto  */
    int32_t block_threads;   /* workgroup size 256/512/1024 of the single-shot and the  *
                              * 64-shot kernels; 0 = automatic                          */
    int32_t lds_bytes;       /* LDS budget of a tile's owned-node accumulator, bytes,    *
                              * <= 163840 (the 64-shot kernel accumulates in FP64 in    *
                              * either precision); 0 = automatic                        */
    int32_t formulation;     /* sem_formulation                                         */
    int32_t scatter;         /* sem_scatter                                             */
} sem_options;

typedef struct {
    int64_t n_elements;
    int64_t n_nodes;
    int32_t p;
    int32_t n_shots;
    int32_t precision;
    int32_t n_sources;       /* after merging sources on the same (node, shot)         */
    int32_t n_receivers;
    int32_t tile_elems;      /* fixed tile size, 0 when tiles are adaptive              */
    int32_t shot_lanes;
    int32_t max_owned_nodes; /* largest owned-node range of a tile                      */
    int32_t tile_items;      /* adaptive cap on own + halo elements per tile            */
    int32_t geometry_on_the_fly; /* 1: geometric factors computed in-kernel per step   */
    int32_t block_threads;   /* threads per workgroup of the step kernel                */
    int64_t n_tiles;
    int64_t halo_elements;   /* sum over tiles of neighbour elements recomputed         */
    int64_t step;            /* steps taken since the last reset                        */
    double dt;
    double dt_stable;        /* 2/sqrt(lambda_max) from power iteration (0 host-only)  */
    double lambda_max;
    double alg_bytes_per_step;  /* algorithmic HBM bytes of one step: per element nq   *
                                 * int32 ids, 3 nq geometric factors and c2; per node *
                                 * dt/M and, per shot, u and v read and written.      *
                                 * SEM_FORM_HEUN: per element nq ids, 8 record words, *
                                 * V read and written (2 nq words each); per node 5   *
                                 * words (U^n, U~ and 1/M-bar read, two U written)    */
    double alg_flops_per_step;
    double setup_seconds;    /* host setup wall time (numbering, reorder, geometry)   */
    double reorder_seconds;  /* part of setup spent on element and node reordering    */
    int32_t max_accum_nodes; /* LDS accumulator slots of the largest tile: its owned   *
                              * nodes, or with 64 shot lanes its owned nodes of two or *
                              * more elements (each tile's owned range lists those     *
                              * first, then the nodes of a single element)             */
    double kernel_bytes_per_step; /* least bytes this context's step kernel reads and   *
                                   * writes (the single-shot kernel computes geometric *
                                   * factors from 8 words per element)                 */
    int32_t n_colours;       /* colours of the greedy element colouring in the element  *
                              * order (Sec. 5; computed for every context)              */
    int32_t scatter;         /* the sem_scatter in use (AUTO resolved)                   */
    int32_t vertices_per_element; /* 4 quadrilaterals, 3 triangles                   */
    double growth_per_step;  /* largest per-step amplification of the time stepper at    *
                              * h^2 lambda_max: 1 for leapfrog below dt_stable; for Heun *
                              * sqrt(1 + (h^2 lambda_max)^2 / 4), above 1 for any h     *
                              * (lambda_max from the leapfrog operator's power iteration)*/
} sem_info;

/* Build the context: validate the mesh, number the GLL nodes, reorder elements and
 * nodes, compute geometric factors, mass and dt, allocate device state (u = v = 0).
 * Errors: INVALID_ARG, BAD_MESH, UNSTABLE_DT (explicit dt too large), HIP, OOM.
 * On error *out is set to NULL and sem_create_error() returns the message. */
int sem_create(const sem_mesh* mesh, const sem_options* opt, sem_ctx** out);

/* Message of the last failed sem_create in this thread. */
const char* sem_create_error(void);

int sem_get_info(const sem_ctx* ctx, sem_info* info);

/* new -> old permutations of the elements [n_elements] and global nodes [n_nodes]
 * (host buffers owned by the caller). Either pointer may be NULL. */
int sem_get_permutations(const sem_ctx* ctx, int32_t* elem_new2old, int32_t* node_new2old);

/* Greedy element colour of every element, ORIGINAL element order, [n_elements] host buffer
 * (Sec. 5: elements are visited in the context's element order and each takes the smallest
 * colour not used by an already-visited element sharing a global node). */
int sem_get_colours(const sem_ctx* ctx, int32_t* colour);

/* Coordinates of the global nodes, original numbering, [n_nodes][2] host buffer. */
int sem_get_node_coords(const sem_ctx* ctx, double* xy);

/* Point sources (Alg. 3): source i sits at the global node nearest to xy[i] (equal
 * distances -> lowest original id), belongs to shot shot[i], and injects a Ricker
 * wavelet r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2, at t_n = n dt. Sources on the
 * same (node, shot) add up. Replaces earlier sources. node_out (may be NULL) receives the
 * snapped original node id of each source. */
int sem_set_sources(sem_ctx* ctx, int32_t n, const double* xy, const int32_t* shot,
                    double f0, double t0, int32_t* node_out);

/* Receivers: the nearest global node to each xy (same tie rule); every shot records u at
 * all receivers after each step. node_out as above. */
int sem_set_receivers(sem_ctx* ctx, int32_t n, const double* xy, int32_t* node_out);

/* Replace the model c^2 ([n_elements] double, original element order): a host array when
 * on_device = 0, a device array (read in stream order on the context stream) when
 * on_device = 1. Keeps dt and re-checks stability: lambda_max(M^-1 K) scales at most with
 * max_e(c2_e / c2ref_e) against the model of the last power iteration, and the power
 * iteration runs again only if that bound leaves dt unproven (then UNSTABLE_DT if dt is
 * too large). Resets the state (u = v = 0). Errors: INVALID_ARG (non-positive or
 * non-finite c2, on_device not 0/1, first-order formulation), NO_DEVICE (on_device = 1 on a
 * host-only context), UNSTABLE_DT, HIP. */
int sem_set_c2(sem_ctx* ctx, const double* c2, int32_t on_device);

/* u = v = 0, step counter = 0. */
int sem_reset(sem_ctx* ctx);

/* Advance nsteps steps. traces_dev (may be NULL) is a device buffer
 * [n_shots][n_receivers][nsteps] of the context precision; column j receives u after
 * step j of this call. Asynchronous on the context stream. */
int sem_run(sem_ctx* ctx, int64_t nsteps, void* traces_dev);

/* One step without recording (sem_run(ctx, 1, NULL)). */
int sem_step(sem_ctx* ctx);

/* Copy the current field out of / into the context: device buffer [n_shots][n_nodes] of
 * the context precision, ORIGINAL node numbering. For V the value is v^{n-1/2}
 * (SEM_FORM_LEAPFROG only; INVALID_ARG for SEM_FORM_HEUN). */
int sem_get_field(sem_ctx* ctx, int32_t which, void* dev);
int sem_set_field(sem_ctx* ctx, int32_t which, const void* dev);

/* One application r = K u of the assembled stiffness (Eq. R with the second-order flux),
 * both device buffers [n_shots][n_nodes] in original numbering. For operator checks. */
int sem_apply_stiffness(sem_ctx* ctx, const void* u_dev, void* r_dev);

/* sem_apply_stiffness without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The permuted input and the result are staged in a static per-device scratch array of
 * 64 MiB (held by every device the library runs on until the process ends), so
 * n_nodes * n_shots * word size must be <= 32 MiB (else INVALID_ARG, nothing launched).
 * Asynchronous on the context stream (no synchronisation). All calls on one device share the
 * scratch: calls that can overlap in time on one device (other streams, other threads, other
 * contexts on the device) race and must be serialised by the caller. */
int sem_apply_stiffness_noalloc(sem_ctx* ctx, const void* u_dev, void* r_dev);

/* Gradient of a loss of the receiver traces with respect to c^2 of every element.
 * Runs the forward from rest for nsteps steps storing (u, v) every ckpt_every steps, then
 * the discrete adjoint backwards segment by segment, recomputing each segment's forward
 * states from its checkpoint. dL_dtraces_dev: device [n_shots][n_receivers][nsteps] of the
 * context precision. grad_c2_dev: device [n_elements] double, original element order,
 * overwritten. Leaves the context reset. */
int sem_adjoint_gradient(sem_ctx* ctx, const void* dL_dtraces_dev, int64_t nsteps,
                         int32_t ckpt_every, double* grad_c2_dev);

/* Wait for all work queued on the context stream. */
int sem_synchronize(sem_ctx* ctx);

/* Position of every cell (cx[i], cy[i]) along the generalized Hilbert curve over a W x H
 * cell grid (the element key of the Hilbert order, Sec. 4.3 step 2). Host arrays. */
int sem_hilbert_index(int64_t W, int64_t H, int64_t n, const int64_t* cx, const int64_t* cy,
                      int64_t* index_out);

/* Launch-configuration autotuner. Times the step kernel of every candidate configuration
 * on this mesh and returns the fastest. Only fields of *base that are zero vary:
 *   n_shots == 1 or triangles: block_threads in {256, 512, 1024} x tile_items in {1, 2}
 *                        workgroup passes (quadrilaterals) or {8, 14, 20} (triangles), a pass
 *                        being 64 / (p+1) (64 / nodes per triangle) elements per wave;
 *   n_shots % 64 == 0:   block_threads in {256, 512} x lds_bytes in {24, 32, 48, 64} KB;
 *   other shot batches:  shot_lanes in {1, 2, 4, 8, 16} (those dividing n_shots).
 * Each candidate runs the full sem_create (setup, dt check), `warmup` untimed steps and
 * `steps` timed steps (HIP events on base->stream, no sources or receivers), then is
 * destroyed. base->device must be a device ordinal. On return *best holds *base with the
 * winning fields filled in and *best_us its time per step; table (may be NULL) receives
 * up to table_cap rows of 5 doubles (block_threads, shot_lanes, lds_bytes, tile_items, us
 * per step, -1 for a candidate whose setup failed) and *n_tried (may be NULL) the number
 * of candidates. Errors: INVALID_ARG, NO_DEVICE (device < 0), or the error of sem_create
 * when no candidate could be built. */
int sem_autotune(const sem_mesh* mesh, const sem_options* base, int32_t warmup, int32_t steps,
                 sem_options* best, double* best_us, double* table, int32_t table_cap,
                 int32_t* n_tried);

/* Description of the last error on this context (never NULL). */
const char* sem_last_error(const sem_ctx* ctx);

/* Free the context and its device memory (synchronises its stream first). */
void sem_destroy(sem_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H_ */
