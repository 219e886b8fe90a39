// api.hip -- the extern "C" boundary: context lifetime, device memory, step driver,
// sources/receivers, field I/O, stiffness apply and the checkpointed adjoint gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "kernels.h"
#include "plan.h"

namespace {

thread_local std::string g_create_error;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

// Scratch of the allocation-free stiffness apply: the permuted input and the result of one
// call, each at most half of it. Every device the library runs on holds its own copy for the
// life of the process; calls on one device share it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct sem_ctx {
    sem::Plan plan;
    sem::MeshIn mesh;                 // pointers valid only during sem_create
    int precision = SEM_F32;
    int S = 1, SL = 1;
    int geo = 0;                      // kernel code of sem::launch_step (0: shot-batch kernel)
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    std::string err;
    size_t wsize = 4;                 // bytes per state word
    // device mesh/tiling
    DevBuf conn, G, c2, dtminv, tile_eb, tile_nb, tile_ns, halo_b, halo, n2o_node, n2o_elem;
    // state
    DevBuf u[2], v;
    int cur = 0;
    int64_t step = 0;
    // sources / receivers (per-tile CSR on device)
    DevBuf src_b, src_loc, src_shot, src_w, rec_b, rec_loc, rec_idx;
    int32_t n_src = 0, n_rec = 0;
    double f0 = 10.0, t0 = 0.1;
    double lambda_max = 0.0, dt_stable = 0.0;
    // the model (new element order) of the last power iteration and its estimate: a later
    // model m is bounded by lambda_max(m) <= max_e(m_e / ref_e) * lambda_max(ref)
    std::vector<double> c2_ref;
    double lambda_ref = 0.0;
    double setup_seconds = 0.0;
    std::vector<DevBuf*> owned;       // every DevBuf to free at destroy
    // first-order system with Heun (SEM_FORM_HEUN): a third U buffer, V at the start and
    // the end of a step ([E][2][nq] each), and 1 / M-bar weighted by 1/c^2
    int formulation = SEM_FORM_LEAPFROG;
    int scatter = SEM_SCATTER_LDS_ATOMIC;
    DevBuf u_next, hv[2], minv_w;
    // the next step's predicted U~ (written by the fused corrector) and whether u[cur ^ 1]
    // holds U~ for the current state (false after any change of state or sources)
    DevBuf u_pred;
    bool heun_pred_valid = false;
    std::vector<DevBuf> extra;        // scratch owned by the adjoint driver
    // global-accumulator scatter (COLOUR, ATOMIC): r [N] (zero between steps), the point
    // lists with new node ids, the element array position -> new element index, and the
    // launch ranges of the element arrays (one per colour; [0, E) for ATOMIC)
    DevBuf racc, src_node, rec_node;
    DevBuf tri_S;                     // triangles: reference matrices [3][nq][nq]
    // 64-shot atomic scatter: owned border nodes per tile, all border nodes, and the
    // receivers at border nodes (receiver index, node)
    DevBuf tile_nbd, border_nodes, brec_idx, brec_node;
    int32_t n_brec = 0;
    bool border = false;
    std::vector<int32_t> elem_slot;
    std::vector<int64_t> ranges;
};

namespace {

#define SEM_HIP(ctx, call)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                       \
            return e_ == hipErrorOutOfMemory ? SEM_ERR_OOM : SEM_ERR_HIP;                         \
        }                                                                                         \
    } while (0)

int fail(sem_ctx* c, int code, const std::string& msg) {
    c->err = msg;
    return code;
}

hipError_t dev_alloc(DevBuf& b, size_t bytes) {
    if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

void dev_free(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename Src>
hipError_t upload(sem_ctx* c, DevBuf& b, const std::vector<Src>& v) {
    hipError_t e = dev_alloc(b, v.size() * sizeof(Src));
    if (e != hipSuccess || v.empty()) return e;
    e = hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(Src), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

// cast a double vector to the context precision and upload
hipError_t upload_real(sem_ctx* c, DevBuf& b, const std::vector<double>& v, double scale = 1.0) {
    if (c->precision == SEM_F64) {
        if (scale == 1.0) return upload(c, b, v);
        std::vector<double> t(v.size());
        for (size_t i = 0; i < v.size(); ++i) t[i] = v[i] * scale;
        return upload(c, b, t);
    }
    std::vector<float> t(v.size());
    for (size_t i = 0; i < v.size(); ++i) t[i] = (float)(v[i] * scale);
    return upload(c, b, t);
}

template <typename T>
sem::StepArgs<T> base_args(sem_ctx* c) {
    sem::StepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    const sem::Plan& P = c->plan;
    a.conn = (const int32_t*)c->conn.p;
    a.G = (const T*)c->G.p;
    a.c2 = (const T*)c->c2.p;
    a.dtminv = (const T*)c->dtminv.p;
    a.E = P.ne;
    a.S = c->S;
    a.conn_bytes = (uint32_t)c->conn.bytes;
    a.G_bytes = (uint32_t)c->G.bytes;
    a.c2_bytes = (uint32_t)c->c2.bytes;
    a.state_bytes = (uint32_t)((size_t)P.nn * c->S * c->wsize);
    // bounds of the buffer-resource reads of dt/M use the same byte count as the state
    a.tile_eb = (const int32_t*)c->tile_eb.p;
    a.tile_nb = (const int32_t*)c->tile_nb.p;
    a.tile_ns = (const int32_t*)c->tile_ns.p;
    a.tile_nbd = c->border ? (const int32_t*)c->tile_nbd.p : nullptr;
    a.halo_b = (const int32_t*)c->halo_b.p;
    a.halo = (const int32_t*)c->halo.p;
    a.n_slices = c->S / c->SL;
    a.lds_own = (P.max_owned + 63) & ~63;   // prefetch chunks are 64 entries
    a.dt = (T)P.dt;
    a.n_rec = c->n_rec;
    a.f0 = c->f0;
    a.t0 = c->t0;
    a.tri_S = (const T*)c->tri_S.p;
    for (int i = 0; i < P.n * P.n; ++i) a.D[i] = (T)P.D[i];
    for (int i = 0; i < P.n; ++i) {
        a.xi[i] = (T)P.xi[i];
        a.w[i] = (T)P.w[i];
    }
    return a;
}

// accumulator bytes of the largest tile: all owned nodes, or (64-shot kernel, FP64
// accumulators in either precision) the owned nodes of two or more elements
size_t lds_bytes(const sem_ctx* c) {
    if (c->geo >= sem::kGeoShots && c->geo < sem::kGeoTri)
        return (size_t)c->plan.max_shared * c->SL * sizeof(double);
    return (size_t)c->plan.max_owned * c->SL * sizeof(double);
}

bool row_kernel(const sem_ctx* c);
bool shots_kernel(const sem_ctx* c);
bool shot_major(const sem_ctx* c);

// One step-kernel launch over all tiles. The row kernel (one shot lane) keeps the state
// shot-major [S][N] and is launched once per shot with every per-shot array offset.
// Global-accumulator step (scatter COLOUR or ATOMIC, one shot): point terms into r, one
// element launch per range (per colour, or all elements), the node pass, then traces.
template <typename T>
int global_launch(sem_ctx* c, const sem::StepArgs<T>& a0) {
    const sem::Plan& P = c->plan;
    sem::StepArgs<T> a = a0;
    a.racc = (T*)c->racc.p;
    a.shot = 0;
    if (a.src_b != nullptr && c->n_src > 0) {
        a.src_node = (const int32_t*)c->src_node.p;
        a.n_src_pts = c->n_src;
    } else {
        a.src_node = nullptr;
    }
    if ((a.inj != nullptr || a.trace != nullptr) && c->n_rec > 0) {
        a.rec_node = (const int32_t*)c->rec_node.p;
        a.rec_idx = (const int32_t*)c->rec_idx.p;
        a.n_rec_pts = c->n_rec;
    }
    if (a.src_node != nullptr || (a.inj != nullptr && c->n_rec > 0))
        SEM_HIP(c, sem::launch_global_points<T>(a, 0, c->stream));
    const int threads = c->geo / 8;
    for (size_t r = 0; r + 1 < c->ranges.size(); ++r) {
        a.e_begin = (int32_t)c->ranges[r];
        a.e_count = (int32_t)(c->ranges[r + 1] - c->ranges[r]);
        SEM_HIP(c, sem::launch_elems<T>(P.p, threads, c->scatter == SEM_SCATTER_ATOMIC, a, c->stream));
    }
    SEM_HIP(c, sem::launch_node_update<T>(a, P.nn, c->stream));
    if (a.trace != nullptr && c->n_rec > 0) SEM_HIP(c, sem::launch_global_points<T>(a, 1, c->stream));
    return SEM_OK;
}

template <typename T>
int launch(sem_ctx* c, const sem::StepArgs<T>& a) {
    if (c->scatter != SEM_SCATTER_LDS_ATOMIC && !shots_kernel(c)) return global_launch<T>(c, a);
    const int64_t nt = (int64_t)c->plan.tile_eb.size() - 1;
    if (c->border) {
        // 64 shots, atomic scatter: border rows of r_out are sums of atomics (modes 1, 2), and
        // border nodes take u_out in a pass after the step launch (mode 0)
        if (a.mode != 0)
            SEM_HIP(c, sem::launch_fill<T>(a.r_out, T(0), c->plan.nn * (int64_t)c->S, c->stream));
        SEM_HIP(c, sem::launch_step<T>(c->plan.p, c->SL, c->geo, nt, lds_bytes(c), a, c->stream));
        if (a.mode == 0)
            SEM_HIP(c, sem::launch_border<T>(a, (const int32_t*)c->border_nodes.p,
                                             (int64_t)c->plan.border_nodes.size(), (const int32_t*)c->brec_idx.p,
                                             (const int32_t*)c->brec_node.p, c->n_brec, c->stream));
        return SEM_OK;
    }
    if (!shot_major(c) || c->S == 1) {
        SEM_HIP(c, sem::launch_step<T>(c->plan.p, c->SL, c->geo, nt, lds_bytes(c), a, c->stream));
        return SEM_OK;
    }
    const int64_t nn = c->plan.nn;
    for (int32_t s = 0; s < c->S; ++s) {
        sem::StepArgs<T> b = a;
        b.n_slices = 1;
        b.shot = s;
        b.state_bytes = (uint32_t)((size_t)nn * sizeof(T));
        const int64_t so = (int64_t)s * nn;
        if (a.u_in) b.u_in = a.u_in + so;
        if (a.u_out) b.u_out = a.u_out + so;
        if (a.v) b.v = a.v + so;
        if (a.r_out) b.r_out = a.r_out + so;
        if (a.u_pair) b.u_pair = a.u_pair + so;
        if (a.trace) b.trace = a.trace + (int64_t)s * a.n_rec * a.trace_cols;
        if (a.inj) b.inj = a.inj + (int64_t)s * a.n_rec * a.inj_cols;
        SEM_HIP(c, sem::launch_step<T>(c->plan.p, c->SL, c->geo, nt, lds_bytes(c), b, c->stream));
    }
    return SEM_OK;
}

// One Heun step of the first-order system: predictor (U, V) -> U~ in u[cur^1], only when
// u[cur^1] does not hold it yet (first step, or after a change of state or sources); then
// the corrector from U~ and (U, V) into u_next, hv[1], fused with the next step's predictor
// into u_pred; those become the state, and u[cur^1] holds the next U~.
template <typename T>
int heun_step(sem_ctx* c, T* trace, int64_t cols, int64_t col) {
    const sem::Plan& P = c->plan;
    sem::HeunArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.conn = (const int32_t*)c->conn.p;
    a.G = (const T*)c->G.p;
    a.minv_w = (const T*)c->minv_w.p;
    a.E = P.ne;
    a.conn_bytes = (uint32_t)c->conn.bytes;
    a.G_bytes = (uint32_t)c->G.bytes;
    a.state_bytes = (uint32_t)((size_t)P.nn * sizeof(T));
    a.tile_eb = (const int32_t*)c->tile_eb.p;
    a.tile_nb = (const int32_t*)c->tile_nb.p;
    a.halo_b = (const int32_t*)c->halo_b.p;
    a.halo = (const int32_t*)c->halo.p;
    a.lds_own = (P.max_owned + 63) & ~63;     // prefetch chunks are 64 entries
    for (int i = 0; i < P.n * P.n; ++i) a.D[i] = (T)P.D[i];
    for (int i = 0; i < P.n; ++i) {
        a.xi[i] = (T)P.xi[i];
        a.w[i] = (T)P.w[i];
    }
    a.f0 = c->f0;
    a.t0 = c->t0;
    if (c->n_src > 0) {
        a.src_b = (const int32_t*)c->src_b.p;
        a.src_loc = (const int32_t*)c->src_loc.p;
        a.src_shot = (const int32_t*)c->src_shot.p;
        a.src_w = (const T*)c->src_w.p;
    }
    const int64_t nt = (int64_t)P.tile_eb.size() - 1;
    const size_t lds = (size_t)P.max_owned * sizeof(double);
    const T h = (T)P.dt;
    a.u0 = (const T*)c->u[c->cur].p;
    a.v0 = (const T*)c->hv[0].p;
    a.h = h;
    if (!c->heun_pred_valid) {
        // predictor: U~ into u[cur ^ 1]
        a.u_out = (T*)c->u[c->cur ^ 1].p;
        a.src_t = (double)c->step * P.dt;
        SEM_HIP(c, sem::launch_heun_stage<T>(P.p, 0, nt, lds, a, c->stream));
    }
    // corrector, fused with the next step's predictor
    a.u1 = (const T*)c->u[c->cur ^ 1].p;
    a.u_out = (T*)c->u_next.p;
    a.v_out = (T*)c->hv[1].p;
    a.u_pred = (T*)c->u_pred.p;
    a.src_t = (double)(c->step + 1) * P.dt;
    if (trace && c->n_rec > 0) {
        a.rec_b = (const int32_t*)c->rec_b.p;
        a.rec_loc = (const int32_t*)c->rec_loc.p;
        a.rec_idx = (const int32_t*)c->rec_idx.p;
        a.trace = trace;
        a.trace_cols = cols;
        a.trace_col = col;
    }
    SEM_HIP(c, sem::launch_heun_stage<T>(P.p, 2, nt, lds, a, c->stream));
    std::swap(c->u[c->cur], c->u_next);
    std::swap(c->u[c->cur ^ 1], c->u_pred);
    std::swap(c->hv[0], c->hv[1]);
    c->heun_pred_valid = true;
    c->step += 1;
    return SEM_OK;
}

// one forward step u[cur] -> u[cur^1]; optional trace column
template <typename T>
int do_step(sem_ctx* c, T* trace, int64_t cols, int64_t col) {
    if (c->formulation == SEM_FORM_HEUN) return heun_step<T>(c, trace, cols, col);
    sem::StepArgs<T> a = base_args<T>(c);
    a.u_in = (const T*)c->u[c->cur].p;
    a.u_out = (T*)c->u[c->cur ^ 1].p;
    a.v = (T*)c->v.p;
    a.mode = 0;
    if (c->n_src > 0) {
        a.src_b = (const int32_t*)c->src_b.p;
        a.src_loc = (const int32_t*)c->src_loc.p;
        a.src_shot = (const int32_t*)c->src_shot.p;
        a.src_w = (const T*)c->src_w.p;
        a.src_t = (double)c->step * c->plan.dt;
    }
    if (trace && c->n_rec > 0) {
        a.rec_b = (const int32_t*)c->rec_b.p;
        a.rec_loc = (const int32_t*)c->rec_loc.p;
        a.rec_idx = (const int32_t*)c->rec_idx.p;
        a.trace = trace;
        a.trace_cols = cols;
        a.trace_col = col;
    }
    int rc = launch<T>(c, a);
    if (rc != SEM_OK) return rc;
    c->cur ^= 1;
    c->step += 1;
    return SEM_OK;
}

template <typename T>
int zero_state(sem_ctx* c) {
    const int64_t n = c->plan.nn * (int64_t)c->S;
    for (int k = 0; k < 2; ++k) SEM_HIP(c, sem::launch_fill<T>((T*)c->u[k].p, T(0), n, c->stream));
    SEM_HIP(c, sem::launch_fill<T>((T*)c->v.p, T(0), n, c->stream));
    if (c->racc.p) SEM_HIP(c, sem::launch_fill<T>((T*)c->racc.p, T(0), c->plan.nn, c->stream));
    if (c->formulation == SEM_FORM_HEUN && c->u_next.p && c->hv[0].p && c->hv[1].p) {
        const int64_t nvq = 2 * (int64_t)c->plan.nq * c->plan.ne;
        SEM_HIP(c, sem::launch_fill<T>((T*)c->u_next.p, T(0), n, c->stream));
        for (int k = 0; k < 2; ++k) SEM_HIP(c, sem::launch_fill<T>((T*)c->hv[k].p, T(0), nvq, c->stream));
    }
    c->cur = 0;
    c->step = 0;
    c->heun_pred_valid = false;
    return SEM_OK;
}

// lambda_max(M^-1 K) by power iteration with the stiffness-apply mode of the step kernel
template <typename T>
int power_iteration(sem_ctx* c, int iters) {
    const int64_t n = c->plan.nn * (int64_t)c->S;
    std::vector<T> x0(n);
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (auto& v : x0) v = (T)U(rng);
    SEM_HIP(c, hipMemcpyAsync(c->u[0].p, x0.data(), n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    DevBuf nrm;
    SEM_HIP(c, dev_alloc(nrm, sizeof(double)));
    auto sumsq = [&](const T* x, double& out) -> int {
        SEM_HIP(c, sem::launch_fill<double>((double*)nrm.p, 0.0, 1, c->stream));
        SEM_HIP(c, sem::launch_sumsq<T>(x, n, (double*)nrm.p, c->stream));
        SEM_HIP(c, hipMemcpyAsync(&out, nrm.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        SEM_HIP(c, hipStreamSynchronize(c->stream));
        return SEM_OK;
    };
    double nx = 0.0;
    int rc = sumsq((const T*)c->u[0].p, nx);
    if (rc) { dev_free(nrm); return rc; }
    SEM_HIP(c, sem::launch_scale<T>((T*)c->u[0].p, 1.0 / std::sqrt(nx), n, c->stream));
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        sem::StepArgs<T> a = base_args<T>(c);
        a.u_in = (const T*)c->u[0].p;
        a.mode = 2;
        a.r_out = (T*)c->u[1].p;
        rc = launch<T>(c, a);
        if (rc) { dev_free(nrm); return rc; }
        double ny = 0.0;
        rc = sumsq((const T*)c->u[1].p, ny);
        if (rc) { dev_free(nrm); return rc; }
        ny = std::sqrt(ny);
        lam = ny / c->plan.dt;                // |dt M^-1 K x| / dt with |x| = 1
        if (!(ny > 0.0)) break;
        SEM_HIP(c, sem::launch_scale<T>((T*)c->u[1].p, 1.0 / ny, n, c->stream));
        std::swap(c->u[0], c->u[1]);
    }
    dev_free(nrm);
    if (!std::isfinite(lam) || lam < 0.0) {
        c->lambda_max = lam;
        c->dt_stable = 0.0;
        return fail(c, SEM_ERR_UNSTABLE_DT, "stiffness apply produced a non-finite eigenvalue estimate");
    }
    c->lambda_max = lam;
    c->dt_stable = lam > 0.0 ? 2.0 / std::sqrt(lam) : INFINITY;
    c->c2_ref = c->plan.c2;
    c->lambda_ref = lam;
    return zero_state<T>(c);
}

// Device address of the scratch array on the context's device (current), looked up once per
// device; the array's name is only a host-side stand-in and is never passed to a kernel.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(sem_ctx* c, void** out) {
    if (c->device < 0 || c->device >= kMaxDevices)
        return fail(c, SEM_ERR_INVALID_ARG, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, SEM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[c->device] = p;
    }
    *out = g_scratch_ptr[c->device];
    return SEM_OK;
}

int check_ctx(const sem_ctx* c) { return c ? SEM_OK : SEM_ERR_INVALID_ARG; }

int need_device(sem_ctx* c) {
    if (c->host_only) return fail(c, SEM_ERR_NO_DEVICE, "context was created host-only (device = -1)");
    return SEM_OK;
}

int set_device(sem_ctx* c) {
    SEM_HIP(c, hipSetDevice(c->device));
    return SEM_OK;
}

bool shots_kernel(const sem_ctx* c) { return c->geo >= sem::kGeoShots && c->geo < sem::kGeoTri; }
bool row_kernel(const sem_ctx* c) { return c->geo > 0 && c->geo < sem::kGeoShots; }
bool tri_kernel(const sem_ctx* c) { return c->geo >= sem::kGeoTri; }
// state [S][N] (shot-major, one launch per shot) instead of [N][S]
bool shot_major(const sem_ctx* c) { return row_kernel(c) || tri_kernel(c); }

// Element arrays in the layout of the context's kernel: the single-shot row kernel reads
// element-major records (node ids [E][nq]; [E][8] = bilinear coefficients, c^2, 0); the
// 64-shot kernel reads element-major ids [E][nq] and factors [E][3 nq + 1] (g11, g12, g22
// per node, then c^2); the shot-batch kernel reads 64-element blocks ([E/64][nq][64] ids,
// [E/64][3][nq][64] factors).
template <typename T>
int upload_geometry(sem_ctx* c) {
    const sem::Plan& P = c->plan;
    const int64_t nq = P.nq, ne = P.ne;
    // the kernels address these arrays with 32-bit byte offsets
    const int64_t ni = (int64_t)(P.p - 1) * (P.p - 1);
    if (tri_kernel(c)) {
        // conn [E + H][nq], record [E + H][4] = c_12, c_23, c_13, c^2 (the coefficients of
        // E_12 = Sxx, E_23, E_13 in K_e / c^2: g11 + g12, -g12, g12 + g22): the E elements in
        // curve order, then a copy of each halo element's row in the order of the halo list
        // (the kernel then finds a halo row without first loading its element index)
        const int64_t nh = (int64_t)P.halo.size(), rows = ne + nh;
        if ((double)rows * nq * 4.0 >= 4294967296.0 || (double)rows * 4 * sizeof(T) >= 4294967296.0)
            return fail(c, SEM_ERR_INVALID_ARG, "element arrays exceed 4 GiB (32-bit buffer offsets)");
        std::vector<int32_t> cb((size_t)rows * nq);
        std::vector<double> gb((size_t)rows * 4);
        for (int64_t k = 0; k < rows; ++k) {
            const int64_t e = c->elem_slot[k < ne ? k : P.halo[k - ne]];
            for (int64_t q = 0; q < nq; ++q) cb[k * nq + q] = P.conn_soa[q * ne + e];
            const double g11 = P.tri_G[e], g12 = P.tri_G[(size_t)ne + e], g22 = P.tri_G[(size_t)2 * ne + e];
            gb[k * 4 + 0] = g11 + g12;
            gb[k * 4 + 1] = -g12;
            gb[k * 4 + 2] = g12 + g22;
            gb[k * 4 + 3] = P.c2[e];
        }
        SEM_HIP(c, upload(c, c->conn, cb));
        SEM_HIP(c, upload_real(c, c->G, gb));
        SEM_HIP(c, upload_real(c, c->tri_S, P.tri_S));
        return SEM_OK;
    }
    const int64_t words = shots_kernel(c) ? 3 * nq + 1 + ni : row_kernel(c) ? 8 : 3 * nq;
    const int64_t n_rec = shots_kernel(c) || row_kernel(c) ? ne : (ne + 63) / 64 * 64;
    if ((double)n_rec * words * sizeof(T) >= 4294967296.0 || (double)n_rec * nq * 4.0 >= 4294967296.0)
        return fail(c, SEM_ERR_INVALID_ARG, "element arrays exceed 4 GiB (32-bit buffer offsets)");
    if (shots_kernel(c)) {
        // record: g11, g12, g22 per node, c2, then dt/M at the (p-1)^2 element-interior
        // nodes (b = 1..p-1 outer, a = 1..p-1 inner)
        const int64_t ni = (int64_t)(P.p - 1) * (P.p - 1), rec = 3 * nq + 1 + ni;
        std::vector<int32_t> cb((size_t)ne * nq);
        std::vector<double> gb((size_t)ne * rec);
        for (int64_t e = 0; e < ne; ++e) {
            for (int64_t q = 0; q < nq; ++q) {
                cb[e * nq + q] = P.conn_soa[q * ne + e];
                for (int64_t k = 0; k < 3; ++k) gb[e * rec + k * nq + q] = P.G_soa[(k * nq + q) * ne + e];
            }
            gb[e * rec + 3 * nq] = P.c2[e];
            for (int b = 1; b < P.p; ++b)
                for (int a2 = 1; a2 < P.p; ++a2) {
                    const int32_t node = P.conn_soa[(int64_t)(a2 + P.n * b) * ne + e];
                    gb[e * rec + 3 * nq + 1 + (b - 1) * (P.p - 1) + (a2 - 1)] = P.minv[node] * P.dt;
                }
        }
        SEM_HIP(c, upload(c, c->conn, cb));
        SEM_HIP(c, upload_real(c, c->G, gb));
        return SEM_OK;
    }
    if (row_kernel(c)) {
        // position k of the element arrays holds new element elem_slot[k] (the curve order,
        // or for the COLOUR scatter the colour classes one after another, each in curve order)
        std::vector<int32_t> cb((size_t)ne * nq);
        std::vector<double> gb((size_t)ne * 8, 0.0);
        for (int64_t k = 0; k < ne; ++k) {
            const int64_t e = c->elem_slot[k];
            for (int64_t q = 0; q < nq; ++q) cb[k * nq + q] = P.conn_soa[q * ne + e];
            for (int64_t j = 0; j < 6; ++j) gb[k * 8 + j] = P.bilin[j * ne + e];
            gb[k * 8 + 6] = P.c2[e];
        }
        SEM_HIP(c, upload(c, c->conn, cb));
        SEM_HIP(c, upload_real(c, c->G, gb));
        return SEM_OK;
    }
    const int64_t nblk = (ne + 63) / 64;
    std::vector<int32_t> cb((size_t)nblk * nq * 64);
    std::vector<double> gb((size_t)nblk * 3 * nq * 64);
    for (int64_t e = 0; e < nblk * 64; ++e) {
        const int64_t src = e < ne ? e : 0, b = e / 64, l = e % 64;
        for (int64_t q = 0; q < nq; ++q) {
            cb[(b * nq + q) * 64 + l] = P.conn_soa[q * ne + src];
            for (int64_t k = 0; k < 3; ++k)
                gb[((b * 3 + k) * nq + q) * 64 + l] = P.G_soa[(k * nq + q) * ne + src];
        }
    }
    SEM_HIP(c, upload(c, c->conn, cb));
    SEM_HIP(c, upload_real(c, c->G, gb));
    return SEM_OK;
}

template <typename T>
int upload_mesh(sem_ctx* c) {
    const sem::Plan& P = c->plan;
    int rc = upload_geometry<T>(c);
    if (rc) return rc;
    SEM_HIP(c, upload_real(c, c->c2, P.c2));
    SEM_HIP(c, upload_real(c, c->dtminv, P.minv, P.dt));
    SEM_HIP(c, upload(c, c->tile_eb, P.tile_eb));
    SEM_HIP(c, upload(c, c->tile_nb, P.tile_nb));
    if (!P.tile_ns.empty()) SEM_HIP(c, upload(c, c->tile_ns, P.tile_ns));
    if (c->border) {
        SEM_HIP(c, upload(c, c->tile_nbd, P.tile_nbd));
        SEM_HIP(c, upload(c, c->border_nodes, P.border_nodes.empty() ? std::vector<int32_t>{0} : P.border_nodes));
    }
    SEM_HIP(c, upload(c, c->halo_b, P.halo_b));
    std::vector<int32_t> h = P.halo;
    if (h.empty()) h.push_back(0);
    SEM_HIP(c, upload(c, c->halo, h));
    SEM_HIP(c, upload(c, c->n2o_node, P.node_new2old));
    std::vector<int32_t> e2o(P.ne);
    for (int64_t k = 0; k < P.ne; ++k) e2o[k] = P.elem_new2old[c->elem_slot[k]];
    SEM_HIP(c, upload(c, c->n2o_elem, e2o));
    const size_t state = (size_t)P.nn * c->S * sizeof(T);
    for (int k = 0; k < 2; ++k) SEM_HIP(c, dev_alloc(c->u[k], state));
    SEM_HIP(c, dev_alloc(c->v, state));
    if (c->scatter != SEM_SCATTER_LDS_ATOMIC) SEM_HIP(c, dev_alloc(c->racc, (size_t)P.nn * sizeof(T)));
    return zero_state<T>(c);
}

// 64 shot lanes (one wave per element) when the batch is a multiple of 64; otherwise one
// lane: the single-shot row kernel, one block per tile and shot
// First-order system: 1 / M-bar with M-bar_nu = sum over (e, q -> nu) of w_q detJ_q / c_e^2
// (Eq. A-bar with M = 1/K, rho = 1), new numbering; V buffers and the third U buffer.
template <typename T>
int setup_heun(sem_ctx* c) {
    const sem::Plan& P = c->plan;
    const int nq = P.nq;
    std::vector<double> mbar(P.nn, 0.0), g11(nq), g12(nq), g22(nq), det(nq);
    for (int64_t e = 0; e < P.ne; ++e) {
        sem::element_geometry(P, c->mesh, e, g11.data(), g12.data(), g22.data(), det.data());
        const double inv_c2 = 1.0 / c->mesh.c2[e];
        for (int b = 0; b < P.n; ++b)
            for (int a = 0; a < P.n; ++a) {
                const int q = a + P.n * b;
                mbar[P.conn0[e * nq + q]] += P.w[a] * P.w[b] * det[q] * inv_c2;
            }
    }
    std::vector<double> inv(P.nn);
    for (int64_t v = 0; v < P.nn; ++v) inv[v] = 1.0 / mbar[P.node_new2old[v]];
    SEM_HIP(c, upload_real(c, c->minv_w, inv));
    const size_t nvq = (size_t)2 * nq * P.ne * sizeof(T);
    for (int k = 0; k < 2; ++k) SEM_HIP(c, dev_alloc(c->hv[k], nvq));
    SEM_HIP(c, dev_alloc(c->u_next, (size_t)P.nn * sizeof(T)));
    SEM_HIP(c, dev_alloc(c->u_pred, (size_t)P.nn * sizeof(T)));
    return zero_state<T>(c);
}

int pick_shot_lanes(int S, int requested) {
    if (requested > 0) return requested;
    return S % 64 == 0 ? 64 : 1;
}

// Adaptive tiles: one workgroup pass covers kBlock / shot_lanes elements; single-shot
// tiles fill exactly one pass, shot batches up to four. The LDS accumulator of the owned
// nodes stays within 64 KB so several workgroups share a CU.
int pick_tile_items(int p, int sl, int row_block, int requested) {
    if (requested > 0) return requested;
    // single shot: one pass of the row kernel; shot batches: four passes of 256 threads
    return sl == 1 ? (64 / (p + 1)) * (row_block / 64) : 4 * sem::kBlock / sl;
}

// Accumulator slots per tile: the LDS accumulator [slots][shot_lanes] fills lds_budget
// bytes (default 64 KB; 64-shot kernel, whose accumulators are FP64: 64 KB with 512
// threads in FP32, 48 KB with 256 threads in FP64, measured on the 512^2 p=4 batch).
int pick_max_owned(int sl, int precision, int lds_budget) {
    (void)precision;
    const int word = 8;                           // accumulators are FP64 in every kernel
    int budget = lds_budget;
    if (budget <= 0) budget = sl == 64 ? (precision == SEM_F64 ? 48 : 64) * 1024 : 65536;
    return budget / (sl * word);
}

// owning tile of a new node id
int64_t tile_of_node(const sem::Plan& P, int32_t v) {
    auto it = std::upper_bound(P.tile_nb.begin(), P.tile_nb.end(), v);
    return (int64_t)(it - P.tile_nb.begin()) - 1;
}

template <typename T>
int set_sources_t(sem_ctx* c, int32_t n, const double* xy, const int32_t* shot, int32_t* node_out) {
    const sem::Plan& P = c->plan;
    const int64_t nt = (int64_t)P.tile_eb.size() - 1;
    struct Ent { int64_t tile; int32_t loc; int32_t shot; double w; };
    std::vector<Ent> ents;
    std::vector<int32_t> near((size_t)std::max(n, 0));
    sem::nearest_nodes(P, n, xy, near.data());
    for (int32_t i = 0; i < n; ++i) {
        const int32_t old = near[i];
        if (node_out) node_out[i] = old;
        const int32_t nw = P.node_old2new[old];
        const int64_t t = tile_of_node(P, nw);
        ents.push_back({t, nw - P.tile_nb[t], shot[i], 1.0});
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
        if (a.tile != b.tile) return a.tile < b.tile;
        if (a.loc != b.loc) return a.loc < b.loc;
        return a.shot < b.shot;
    });
    std::vector<Ent> merged;
    for (const Ent& e : ents) {
        if (!merged.empty() && merged.back().tile == e.tile && merged.back().loc == e.loc &&
            merged.back().shot == e.shot)
            merged.back().w += e.w;
        else
            merged.push_back(e);
    }
    std::vector<int32_t> b(nt + 1, 0), loc, sh, node;
    std::vector<double> w;
    for (const Ent& e : merged) {
        b[e.tile + 1]++;
        loc.push_back(e.loc);
        sh.push_back(e.shot);
        w.push_back(e.w);
        node.push_back(P.tile_nb[e.tile] + e.loc);
    }
    for (int64_t t = 0; t < nt; ++t) b[t + 1] += b[t];
    c->n_src = (int32_t)merged.size();
    if (c->host_only) return SEM_OK;
    SEM_HIP(c, upload(c, c->src_b, b));
    SEM_HIP(c, upload(c, c->src_loc, loc));
    SEM_HIP(c, upload(c, c->src_shot, sh));
    SEM_HIP(c, upload_real(c, c->src_w, w));
    SEM_HIP(c, upload(c, c->src_node, node));
    return SEM_OK;
}

template <typename T>
int set_receivers_t(sem_ctx* c, int32_t n, const double* xy, int32_t* node_out) {
    const sem::Plan& P = c->plan;
    const int64_t nt = (int64_t)P.tile_eb.size() - 1;
    struct Ent { int64_t tile; int32_t loc; int32_t r; };
    std::vector<Ent> ents;
    std::vector<int32_t> near((size_t)std::max(n, 0));
    sem::nearest_nodes(P, n, xy, near.data());
    for (int32_t i = 0; i < n; ++i) {
        const int32_t old = near[i];
        if (node_out) node_out[i] = old;
        const int32_t nw = P.node_old2new[old];
        const int64_t t = tile_of_node(P, nw);
        ents.push_back({t, nw - P.tile_nb[t], i});
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.tile < b.tile; });
    std::vector<int32_t> b(nt + 1, 0), loc, idx, node;
    for (const Ent& e : ents) {
        b[e.tile + 1]++;
        loc.push_back(e.loc);
        idx.push_back(e.r);
        node.push_back(P.tile_nb[e.tile] + e.loc);
    }
    for (int64_t t = 0; t < nt; ++t) b[t + 1] += b[t];
    c->n_rec = n;
    if (c->host_only) return SEM_OK;
    SEM_HIP(c, upload(c, c->rec_b, b));
    SEM_HIP(c, upload(c, c->rec_loc, loc.empty() ? std::vector<int32_t>{0} : loc));
    SEM_HIP(c, upload(c, c->rec_idx, idx.empty() ? std::vector<int32_t>{0} : idx));
    SEM_HIP(c, upload(c, c->rec_node, node.empty() ? std::vector<int32_t>{0} : node));
    if (c->border) {
        std::vector<int32_t> bi, bn;
        for (const Ent& e : ents)
            if (e.loc >= P.tile_ns[e.tile] && e.loc < P.tile_ns[e.tile] + P.tile_nbd[e.tile]) {
                bi.push_back(e.r);
                bn.push_back(P.tile_nb[e.tile] + e.loc);
            }
        c->n_brec = (int32_t)bi.size();
        SEM_HIP(c, upload(c, c->brec_idx, bi.empty() ? std::vector<int32_t>{0} : bi));
        SEM_HIP(c, upload(c, c->brec_node, bn.empty() ? std::vector<int32_t>{0} : bn));
    }
    return SEM_OK;
}

template <typename T>
int run_t(sem_ctx* c, int64_t nsteps, void* traces) {
    for (int64_t j = 0; j < nsteps; ++j) {
        int rc = do_step<T>(c, (T*)traces, nsteps, j);
        if (rc) return rc;
    }
    return SEM_OK;
}

// r = K u through staging buffers tin, tout ([S][N] new numbering, context precision):
// permute u in, one stiffness launch (mode 1), permute r out. Asynchronous on the stream.
template <typename T>
int apply_into(sem_ctx* c, const void* u_dev, void* r_dev, void* tin, void* tout) {
    const int64_t N = c->plan.nn;
    SEM_HIP(c, sem::launch_nodes_from_original<T>((const T*)u_dev, (T*)tin, (const int32_t*)c->n2o_node.p, N,
                                                  c->S, shot_major(c), c->stream));
    sem::StepArgs<T> a = base_args<T>(c);
    a.u_in = (const T*)tin;
    a.mode = 1;
    a.r_out = (T*)tout;
    int rc = launch<T>(c, a);
    if (rc) return rc;
    SEM_HIP(c, sem::launch_nodes_to_original<T>((const T*)tout, (T*)r_dev, (const int32_t*)c->n2o_node.p, N,
                                                c->S, shot_major(c), c->stream));
    return SEM_OK;
}

template <typename T>
int apply_t(sem_ctx* c, const void* u_dev, void* r_dev) {
    DevBuf tin, tout;
    const size_t bytes = (size_t)c->plan.nn * c->S * sizeof(T);
    SEM_HIP(c, dev_alloc(tin, bytes));
    hipError_t e = dev_alloc(tout, bytes);
    if (e != hipSuccess) { dev_free(tin); SEM_HIP(c, e); }
    int rc = apply_into<T>(c, u_dev, r_dev, tin.p, tout.p);
    if (rc == SEM_OK) {
        const hipError_t h = hipStreamSynchronize(c->stream);
        if (h != hipSuccess) rc = fail(c, SEM_ERR_HIP, hipGetErrorString(h));
    }
    dev_free(tin);
    dev_free(tout);
    return rc;
}

// Forward with checkpoints, then the adjoint recurrence backwards segment by segment.
// The adjoint state w^j is advanced by the same step kernel with the trace gradient
// injected at the receivers (amplitude dL/dd[s][r][N-1-j] / dt^2); while it gathers
// w^j for its stiffness apply, it also gathers u^{N-j} from the recomputed segment and
// accumulates (Khat_e w^j_e) . u^{N-j}_e per element, which is mu^{n+1} Khat_e u^n with
// n = N - j. The gradient is -dt^2 times that sum.
template <typename T>
int adjoint_t(sem_ctx* c, const void* dL, int64_t N, int32_t C, double* grad_out) {
    const sem::Plan& P = c->plan;
    const int64_t nnS = P.nn * (int64_t)c->S;
    const size_t sb = (size_t)nnS * sizeof(T);
    const int64_t nck = (N + C - 1) / C;
    std::vector<DevBuf> ck_u(nck), ck_v(nck), seg(C);
    DevBuf w[2], vw, acc;
    auto cleanup = [&]() {
        for (auto& b : ck_u) dev_free(b);
        for (auto& b : ck_v) dev_free(b);
        for (auto& b : seg) dev_free(b);
        dev_free(w[0]); dev_free(w[1]); dev_free(vw); dev_free(acc);
    };
    int rc = SEM_OK;
#define ADJ_HIP(call)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            cleanup();                                                                            \
            c->err = std::string(#call) + ": " + hipGetErrorString(e_);                           \
            return e_ == hipErrorOutOfMemory ? SEM_ERR_OOM : SEM_ERR_HIP;                         \
        }                                                                                         \
    } while (0)
    for (int64_t k = 0; k < nck; ++k) {
        ADJ_HIP(dev_alloc(ck_u[k], sb));
        ADJ_HIP(dev_alloc(ck_v[k], sb));
    }
    for (int32_t i = 0; i < C; ++i) ADJ_HIP(dev_alloc(seg[i], sb));
    ADJ_HIP(dev_alloc(w[0], sb));
    ADJ_HIP(dev_alloc(w[1], sb));
    ADJ_HIP(dev_alloc(vw, sb));
    ADJ_HIP(dev_alloc(acc, (size_t)P.ne * sizeof(double)));

    // forward from rest, checkpoint (u^{kC}, v^{kC-1/2})
    rc = zero_state<T>(c);
    if (rc) { cleanup(); return rc; }
    for (int64_t k = 0; k < nck; ++k) {
        ADJ_HIP(hipMemcpyAsync(ck_u[k].p, c->u[c->cur].p, sb, hipMemcpyDeviceToDevice, c->stream));
        ADJ_HIP(hipMemcpyAsync(ck_v[k].p, c->v.p, sb, hipMemcpyDeviceToDevice, c->stream));
        const int64_t steps = std::min<int64_t>(C, N - k * C);
        for (int64_t i = 0; i < steps; ++i) {
            rc = do_step<T>(c, nullptr, 0, 0);
            if (rc) { cleanup(); return rc; }
        }
    }
    ADJ_HIP(sem::launch_fill<T>((T*)w[0].p, T(0), nnS, c->stream));
    ADJ_HIP(sem::launch_fill<T>((T*)w[1].p, T(0), nnS, c->stream));
    ADJ_HIP(sem::launch_fill<T>((T*)vw.p, T(0), nnS, c->stream));
    ADJ_HIP(sem::launch_fill<double>((double*)acc.p, 0.0, P.ne, c->stream));
    int wc = 0;
    const T inv_dt2 = (T)(1.0 / (P.dt * P.dt));
    auto adjoint_step = [&](int64_t j, const T* upair) -> int {
        sem::StepArgs<T> a = base_args<T>(c);
        a.u_in = (const T*)w[wc].p;
        a.u_out = (T*)w[wc ^ 1].p;
        a.v = (T*)vw.p;
        a.mode = 0;
        if (c->n_rec > 0) {
            a.rec_b = (const int32_t*)c->rec_b.p;
            a.rec_loc = (const int32_t*)c->rec_loc.p;
            a.rec_idx = (const int32_t*)c->rec_idx.p;
            a.inj = (const T*)dL;
            a.inj_cols = N;
            a.inj_col = N - 1 - j;
            a.inj_scale = inv_dt2;
        }
        if (upair) {
            a.u_pair = upair;
            a.grad = (double*)acc.p;
        }
        int r = launch<T>(c, a);
        wc ^= 1;
        return r;
    };
    rc = adjoint_step(0, nullptr);                  // w^0 = 0 pairs with nothing
    if (rc) { cleanup(); return rc; }
    // segments last to first; segment k holds u^{kC} .. u^{kC+C-1}
    for (int64_t k = nck - 1; k >= 0; --k) {
        const int64_t n0 = k * C;
        const int64_t n1 = std::min<int64_t>(n0 + C - 1, N - 1);   // last state needed
        ADJ_HIP(hipMemcpyAsync(seg[0].p, ck_u[k].p, sb, hipMemcpyDeviceToDevice, c->stream));
        ADJ_HIP(hipMemcpyAsync(c->v.p, ck_v[k].p, sb, hipMemcpyDeviceToDevice, c->stream));
        for (int64_t n = n0; n < n1; ++n) {         // u^{n+1} from u^n
            sem::StepArgs<T> a = base_args<T>(c);
            a.u_in = (const T*)seg[n - n0].p;
            a.u_out = (T*)seg[n - n0 + 1].p;
            a.v = (T*)c->v.p;
            a.mode = 0;
            if (c->n_src > 0) {
                a.src_b = (const int32_t*)c->src_b.p;
                a.src_loc = (const int32_t*)c->src_loc.p;
                a.src_shot = (const int32_t*)c->src_shot.p;
                a.src_w = (const T*)c->src_w.p;
                a.src_t = (double)n * P.dt;
            }
            rc = launch<T>(c, a);
            if (rc) { cleanup(); return rc; }
        }
        for (int64_t n = n1; n >= std::max<int64_t>(n0, 1); --n) {
            rc = adjoint_step(N - n, (const T*)seg[n - n0].p);
            if (rc) { cleanup(); return rc; }
        }
    }
    ADJ_HIP(sem::launch_grad_to_original((const double*)acc.p, grad_out, (const int32_t*)c->n2o_elem.p,
                                         P.ne, -P.dt * P.dt, c->stream));
    ADJ_HIP(hipStreamSynchronize(c->stream));
    cleanup();
#undef ADJ_HIP
    return zero_state<T>(c);
}

}  // namespace

extern "C" {

const char* sem_create_error(void) { return g_create_error.c_str(); }

int sem_create(const sem_mesh* mesh, const sem_options* opt, sem_ctx** out) {
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return SEM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (!mesh || !opt) { g_create_error = "mesh or options is NULL"; return SEM_ERR_INVALID_ARG; }
    if (opt->precision != SEM_F32 && opt->precision != SEM_F64) {
        g_create_error = "precision must be SEM_F32 or SEM_F64";
        return SEM_ERR_INVALID_ARG;
    }
    if (opt->n_shots < 1) { g_create_error = "n_shots must be >= 1"; return SEM_ERR_INVALID_ARG; }
    if (opt->p < 1 || opt->p > sem::kMaxP) { g_create_error = "p must be in 1..7"; return SEM_ERR_INVALID_ARG; }
    if (opt->tile_elems < 0 || opt->shot_lanes < 0) {
        g_create_error = "tile_elems and shot_lanes must be >= 0";
        return SEM_ERR_INVALID_ARG;
    }
    if (opt->device >= 0 && opt->node_order != SEM_NODES_FIRST_TOUCH) {
        g_create_error = "device contexts need node_order = SEM_NODES_FIRST_TOUCH (owned node ranges)";
        return SEM_ERR_INVALID_ARG;
    }
    sem_ctx* c = new (std::nothrow) sem_ctx();
    if (!c) { g_create_error = "host allocation failed"; return SEM_ERR_OOM; }
    const auto t0 = std::chrono::steady_clock::now();
    c->precision = opt->precision;
    c->wsize = opt->precision == SEM_F64 ? 8 : 4;
    c->S = opt->n_shots;
    const int nvpe = mesh->vertices_per_element == 0 ? 4 : mesh->vertices_per_element;
    if (nvpe != 3 && nvpe != 4) {
        g_create_error = "vertices_per_element must be 0 or 4 (quadrilaterals) or 3 (triangles)";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    // triangles run one shot per launch of the triangle kernel
    c->SL = nvpe == 3 ? (opt->shot_lanes > 1 ? -1 : 1) : pick_shot_lanes(c->S, opt->shot_lanes);
    if (c->SL < 1 || c->SL > 64 || (c->SL & (c->SL - 1)) || c->S % c->SL) {
        g_create_error = "shot_lanes must be a power of two <= 64 dividing n_shots";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    c->device = opt->device;
    c->host_only = opt->device < 0;
    c->stream = (hipStream_t)opt->stream;
    sem::MeshIn m;
    m.nv = mesh->n_vertices;
    m.ne = mesh->n_elements;
    m.vxy = mesh->vxy;
    m.quad = mesh->quad;
    m.c2 = mesh->c2;
    m.nvpe = nvpe;
    c->mesh = m;                                  // valid until sem_create returns
    if (nvpe == 3 && opt->formulation != SEM_FORM_LEAPFROG) {
        g_create_error = "triangles run the second-order leapfrog formulation";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    if (opt->formulation != SEM_FORM_LEAPFROG && opt->formulation != SEM_FORM_HEUN) {
        g_create_error = "unknown formulation";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    if (opt->formulation == SEM_FORM_HEUN && c->S != 1) {
        g_create_error = "the first-order (Heun) formulation runs a single shot";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    c->formulation = opt->formulation;
    if (opt->scatter < SEM_SCATTER_AUTO || opt->scatter > SEM_SCATTER_ATOMIC) {
        g_create_error = "unknown scatter";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    // AUTO: owner-tile LDS accumulation, measured fastest for every kernel (colour passes
    // and global atomics both move r through L2 and HBM)
    c->scatter = opt->scatter == SEM_SCATTER_AUTO ? SEM_SCATTER_LDS_ATOMIC : opt->scatter;
    const bool shots64 = c->S % 64 == 0 && c->SL == 64;
    if (c->scatter != SEM_SCATTER_LDS_ATOMIC &&
        (opt->formulation != SEM_FORM_LEAPFROG || nvpe != 4 ||
         !(c->S == 1 || (shots64 && c->scatter == SEM_SCATTER_ATOMIC)))) {
        g_create_error = "COLOUR runs the single-shot leapfrog step on quadrilaterals, ATOMIC that step or "
                         "batches of 64-shot lanes";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    c->border = shots64 && c->scatter == SEM_SCATTER_ATOMIC;
    sem::PlanOptions po;
    po.p = opt->p;
    po.elem_order = opt->elem_order;
    po.node_order = opt->node_order;
    po.seed = opt->seed;
    po.dt = opt->dt;
    po.cfl = opt->cfl;
    po.tile_elems = opt->tile_elems;
    // measured on the layered 1024^2 p=4 mesh (FP64 LDS accumulators): 512 threads x 1 pass
    // in both precisions
    // triangles default to 256 threads (on the 250k-triangle p = 5 mesh 256 threads with
    // 240-element tiles ran 2.5% (FP32) and 4.4% (FP64) faster than 512 with 336)
    const int row_block = opt->block_threads > 0 ? opt->block_threads : (nvpe == 3 ? 256 : 512);
    if (row_block != 256 && row_block != 512 && row_block != 1024) {
        g_create_error = "block_threads must be 256, 512 or 1024";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    // passes of the row kernel whose loads are batched: enough to cover one tile, <= 4
    const int epb = (64 / (opt->p + 1)) * (row_block / 64);
    const int max_np = row_block == 256 ? 4 : (row_block == 512 ? 2 : 1);
    if (opt->lds_bytes < 0 || opt->lds_bytes > 160 * 1024) {
        g_create_error = "lds_bytes must be in 0..163840";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    po.tile_items = pick_tile_items(opt->p, c->SL, row_block, opt->tile_items);
    if (opt->tile_items <= 0 && c->SL == 1) po.tile_items = epb;
    if (nvpe == 3 && opt->tile_items <= 0) {
        // triangles: tiles of about 240 own + halo elements in whole workgroup passes of
        // 64 / nq elements per wave (twenty passes with 256 threads at p = 5; measured there
        // against 96 and 168: 3% and 1% faster in FP32, 4% and 1% in FP64), and never more owned
        // nodes than the LDS of the resident workgroups allows (the cap below)
        const int epb_tri = (64 / sem::tri_nq(opt->p)) * (row_block / 64);
        po.tile_items = std::max(1, (240 + epb_tri / 2) / epb_tri) * epb_tri;
    }
    // 64 shots: tiles are bounded by the LDS accumulator, not by an element count
    if (opt->tile_items <= 0 && c->SL == 64) po.tile_items = 1 << 20;
    int np = 1;
    while (np < max_np && np * epb < (opt->tile_elems > 0 ? opt->tile_elems : po.tile_items)) np *= 2;
    po.max_owned = pick_max_owned(c->SL, opt->precision, opt->lds_bytes);
    if (nvpe == 3 && opt->lds_bytes <= 0) {
        // triangles: bound a tile's owned nodes so that the workgroups the registers allow on
        // a CU (p = 5: FP32 88 VGPRs, 20 waves a CU; FP64 113, 16 waves) also fit its 160 KB of
        // LDS: on the 250k-triangle mesh, FP32 tiles one pass past that bound ran 38% slower
        const int per_cu = std::max(1, (opt->precision == SEM_F64 ? 16 : 20) / (row_block / 64));
        const size_t word = opt->precision == SEM_F64 ? 8 : 4;
        const size_t stage = sem::tri_lds_bytes(opt->p, row_block, 0, word);
        const size_t budget = 163840 / (size_t)per_cu;
        const int cap = budget > stage ? (int)((budget - stage) / (8 + 3 * word)) & ~63 : 0;
        po.max_owned = std::min(po.max_owned, cap);
    }
    po.split_single = c->S > 1 && c->SL == 64;
    po.border = c->border;
    if (po.max_owned < 1) {
        g_create_error = "lds_bytes too small for one owned node";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    // one shot lane: row kernel with in-kernel geometry (shot-major state, a block per tile
    // and shot); 64 shot lanes: one wave per element
    if (nvpe == 3) c->geo = sem::kGeoTri + row_block;
    else if (c->SL == 1) c->geo = row_block * 8 + np;
    // 64 shots: FP32 512 threads, FP64 256 (p = 4: about 100 VGPRs in FP32, 170 in FP64)
    else if (c->SL == 64)
        c->geo = sem::kGeoShots +
                 (opt->block_threads > 0 ? row_block : (opt->precision == SEM_F64 ? 256 : 512));
    else c->geo = 0;
    int code = SEM_OK;
    std::string err;
    try {
        err = sem::build_plan(m, po, c->plan, code);
    } catch (const std::bad_alloc&) {
        err = "host allocation failed during setup";
        code = SEM_ERR_OOM;
    } catch (const std::exception& ex) {
        err = ex.what();
        code = SEM_ERR_INVALID_ARG;
    }
    if (!err.empty()) {
        g_create_error = err;
        delete c;
        return code;
    }
    {
        const sem::Plan& P = c->plan;
        c->elem_slot.resize(P.ne);
        std::iota(c->elem_slot.begin(), c->elem_slot.end(), 0);
        c->ranges = {0, P.ne};
        if (c->scatter == SEM_SCATTER_COLOUR) {
            // colour classes one after another, each in the element (curve) order
            std::stable_sort(c->elem_slot.begin(), c->elem_slot.end(),
                             [&](int32_t x, int32_t y) { return P.colour[x] < P.colour[y]; });
            c->ranges.assign(P.n_colours + 1, 0);
            for (int64_t k = 0; k < P.ne; ++k) c->ranges[P.colour[k] + 1]++;
            for (int32_t k = 0; k < P.n_colours; ++k) c->ranges[k + 1] += c->ranges[k];
        }
    }
    c->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!c->host_only) {
        // LDS of the largest tile in the kernel this context launches
        const int64_t lds_own = (c->plan.max_owned + 63) & ~63;
        size_t need = lds_bytes(c);
        if (c->formulation == SEM_FORM_HEUN)
            need = sem::heun_lds_bytes(opt->p, 2, lds_own, c->wsize);
        else if (tri_kernel(c))
            need = sem::tri_lds_bytes(opt->p, row_block, lds_own, c->wsize);
        else if (row_kernel(c))
            need = sem::rows_lds_bytes(opt->p, row_block, lds_own, c->wsize);
        if (need > sem::kMaxLds) {
            g_create_error = "the largest tile needs " + std::to_string(need) +
                             " bytes of LDS, more than the 160 KB of a workgroup (use smaller "
                             "tile_elems or tile_items)";
            delete c;
            return SEM_ERR_INVALID_ARG;
        }
    }
    if (!c->host_only && (double)c->plan.nn * c->S * c->wsize >= 4294967296.0) {
        g_create_error = "n_nodes * n_shots * word size must stay below 4 GiB (32-bit buffer offsets)";
        delete c;
        return SEM_ERR_INVALID_ARG;
    }
    if (!c->host_only) {
        int rc = set_device(c);
        void* scratch_ptr = nullptr;
        if (rc == SEM_OK) rc = scratch_address(c, &scratch_ptr);
        if (rc == SEM_OK) rc = c->precision == SEM_F64 ? upload_mesh<double>(c) : upload_mesh<float>(c);
        if (rc == SEM_OK && c->formulation == SEM_FORM_HEUN)
            rc = c->precision == SEM_F64 ? setup_heun<double>(c) : setup_heun<float>(c);
        if (rc == SEM_OK) rc = c->precision == SEM_F64 ? power_iteration<double>(c, 60)
                                                       : power_iteration<float>(c, 60);
        if (rc == SEM_OK && c->plan.dt_from_stability) {
            // triangles: the node-spacing rule does not bound the spectrum of the element, so
            // the default dt is 0.6 of the estimated leapfrog limit
            c->plan.dt = 0.6 * c->dt_stable;
            rc = upload_real(c, c->dtminv, c->plan.minv, c->plan.dt) == hipSuccess ? SEM_OK : SEM_ERR_HIP;
            if (rc) c->err = "upload of dt / M failed";
        }
        if (rc == SEM_OK && !(c->plan.dt < c->dt_stable)) {
            rc = SEM_ERR_UNSTABLE_DT;
            c->err = "dt = " + std::to_string(c->plan.dt) + " exceeds the stability limit " +
                     std::to_string(c->dt_stable);
        }
        if (rc != SEM_OK) {
            g_create_error = c->err;
            sem_destroy(c);
            return rc;
        }
    }
    *out = c;
    return SEM_OK;
}

int sem_get_info(const sem_ctx* c, sem_info* info) {
    if (!c || !info) return SEM_ERR_INVALID_ARG;
    const sem::Plan& P = c->plan;
    std::memset(info, 0, sizeof(*info));
    info->n_elements = P.ne;
    info->n_nodes = P.nn;
    info->p = P.p;
    info->n_shots = c->S;
    info->precision = c->precision;
    info->n_sources = c->n_src;
    info->n_receivers = c->n_rec;
    info->tile_elems = P.tile_elems;
    info->shot_lanes = c->SL;
    info->max_owned_nodes = P.max_owned;
    info->tile_items = P.tile_items;
    info->geometry_on_the_fly = row_kernel(c) ? 1 : 0;
    info->block_threads = tri_kernel(c)     ? c->geo - sem::kGeoTri
                          : shots_kernel(c) ? c->geo - sem::kGeoShots
                          : row_kernel(c)   ? c->geo / 8
                                            : sem::kBlock;
    info->vertices_per_element = P.nvpe;
    info->n_tiles = P.tile_eb.empty() ? 0 : (int64_t)P.tile_eb.size() - 1;
    info->halo_elements = (int64_t)P.halo.size();
    info->step = c->step;
    info->dt = P.dt;
    info->dt_stable = c->dt_stable;
    info->lambda_max = c->lambda_max;
    const double w = (double)c->wsize, nq = (double)P.nq;
    // algorithmic bytes of the method: per element nq node indices, 3 nq stored
    // geometric factors and c2; per node dt/M plus read u, v and write u, v per shot
    const double per_node = (double)P.nn * (w + 4.0 * w * c->S);
    info->alg_bytes_per_step = (double)P.ne * (nq * 4.0 + (3.0 * nq + 1.0) * w) + per_node;
    // what this context's kernel reads at least: the row kernel keeps one 8-word record
    // per element (6 bilinear-map coefficients, c2, padding) instead of stored factors
    // (64-shot kernel: stored factors, c2 and dt/M of the (p-1)^2 element-interior nodes)
    const double elem_words = row_kernel(c) ? 8.0
                              : 3.0 * nq + 1.0 + (shots_kernel(c) ? (P.p - 1.0) * (P.p - 1.0) : 0.0);
    info->kernel_bytes_per_step = (double)P.ne * (nq * 4.0 + elem_words * w) + per_node;
    // global accumulator: every node's r written at least once by the element launches,
    // then read and cleared by the node pass
    if (c->scatter != SEM_SCATTER_LDS_ATOMIC) info->kernel_bytes_per_step += (double)P.nn * 3.0 * w;
    const double n = (double)P.n;
    info->alg_flops_per_step = (double)P.ne * c->S * (8.0 * n * n * n + 7.0 * n * n) +
                               (double)P.nn * c->S * 4.0;
    if (tri_kernel(c)) {
        // affine triangles: per element nq ids, 3 geometric factors and c^2; per node as above;
        // three reference-matrix rows per local node: 6 nq^2 flops and the combination
        info->alg_bytes_per_step = (double)P.ne * (nq * 4.0 + 4.0 * w) + per_node;
        info->kernel_bytes_per_step = info->alg_bytes_per_step;
        info->alg_flops_per_step = (double)P.ne * c->S * (6.0 * nq * nq + 6.0 * nq) + (double)P.nn * c->S * 4.0;
    }
    if (c->formulation == SEM_FORM_HEUN) {
        // one launch per step (the corrector fused with the next predictor); per element:
        // ids and the 8-word record, V^n read and V^{n+1} written (2 nq words each); per
        // node: U^n and U~ read, U^{n+1} and the next U~ written, 1/M-bar read
        info->alg_bytes_per_step = (double)P.ne * (nq * 4.0 + 8.0 * w + 2.0 * 2.0 * nq * w) +
                                   (double)P.nn * 5.0 * w;
        info->kernel_bytes_per_step = info->alg_bytes_per_step;
        info->alg_flops_per_step *= 2.0;
    }
    info->setup_seconds = c->setup_seconds;
    info->reorder_seconds = P.reorder_seconds;
    info->max_accum_nodes = P.tile_ns.empty() ? P.max_owned : P.max_shared;
    info->n_colours = P.n_colours;
    info->scatter = c->scatter;
    info->growth_per_step = 1.0;
    if (c->formulation == SEM_FORM_HEUN && c->lambda_max > 0.0) {
        // Heun on y' = i w y: |1 + z + z^2 / 2|^2 = 1 + th^4 / 4 with z = i th, th = h w
        const double th2 = P.dt * P.dt * c->lambda_max;
        info->growth_per_step = std::sqrt(1.0 + 0.25 * th2 * th2);
    }
    return SEM_OK;
}

int sem_get_permutations(const sem_ctx* c, int32_t* e, int32_t* n) {
    if (!c) return SEM_ERR_INVALID_ARG;
    if (e) std::memcpy(e, c->plan.elem_new2old.data(), c->plan.ne * sizeof(int32_t));
    if (n) std::memcpy(n, c->plan.node_new2old.data(), c->plan.nn * sizeof(int32_t));
    return SEM_OK;
}

int sem_get_colours(const sem_ctx* c, int32_t* colour) {
    if (!c || !colour) return SEM_ERR_INVALID_ARG;
    for (int64_t k = 0; k < c->plan.ne; ++k) colour[c->plan.elem_new2old[k]] = c->plan.colour[k];
    return SEM_OK;
}

int sem_get_node_coords(const sem_ctx* c, double* xy) {
    if (!c || !xy) return SEM_ERR_INVALID_ARG;
    std::memcpy(xy, c->plan.node_xy.data(), c->plan.nn * 2 * sizeof(double));
    return SEM_OK;
}

int sem_set_sources(sem_ctx* c, int32_t n, const double* xy, const int32_t* shot, double f0, double t0,
                    int32_t* node_out) {
    if (!c) return SEM_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!xy || !shot))) return fail(c, SEM_ERR_INVALID_ARG, "bad source arrays");
    for (int32_t i = 0; i < n; ++i)
        if (shot[i] < 0 || shot[i] >= c->S) return fail(c, SEM_ERR_INVALID_ARG, "source shot out of range");
    if (!(f0 > 0.0)) return fail(c, SEM_ERR_INVALID_ARG, "f0 must be positive");
    if (c->plan.tile_eb.empty()) return fail(c, SEM_ERR_INVALID_ARG, "no tiling (node_order ORIGINAL)");
    c->f0 = f0;
    c->t0 = t0;
    if (!c->host_only) { int rc = set_device(c); if (rc) return rc; }
    c->heun_pred_valid = false;
    return c->precision == SEM_F64 ? set_sources_t<double>(c, n, xy, shot, node_out)
                                   : set_sources_t<float>(c, n, xy, shot, node_out);
}

int sem_set_receivers(sem_ctx* c, int32_t n, const double* xy, int32_t* node_out) {
    if (!c) return SEM_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && !xy)) return fail(c, SEM_ERR_INVALID_ARG, "bad receiver arrays");
    if (c->plan.tile_eb.empty()) return fail(c, SEM_ERR_INVALID_ARG, "no tiling (node_order ORIGINAL)");
    if (!c->host_only) { int rc = set_device(c); if (rc) return rc; }
    return c->precision == SEM_F64 ? set_receivers_t<double>(c, n, xy, node_out)
                                   : set_receivers_t<float>(c, n, xy, node_out);
}

int sem_set_c2(sem_ctx* c, const double* c2, int32_t on_device) {
    if (!c || !c2) return SEM_ERR_INVALID_ARG;
    if (c->formulation == SEM_FORM_HEUN)
        return fail(c, SEM_ERR_INVALID_ARG, "sem_set_c2 is not available for the first-order formulation");
    if (on_device != 0 && on_device != 1) return fail(c, SEM_ERR_INVALID_ARG, "on_device must be 0 or 1");
    const int64_t ne = c->plan.ne;
    std::vector<double> host;
    if (on_device) {
        int rc = need_device(c);
        if (rc) return rc;
        rc = set_device(c);
        if (rc) return rc;
        host.resize((size_t)ne);
        // stream-ordered after the caller's work on the context stream
        SEM_HIP(c, hipMemcpyAsync(host.data(), c2, (size_t)ne * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        SEM_HIP(c, hipStreamSynchronize(c->stream));
        c2 = host.data();
    }
    for (int64_t e = 0; e < ne; ++e)
        if (!(c2[e] > 0.0) || !std::isfinite(c2[e])) return fail(c, SEM_ERR_INVALID_ARG, "c2 must be positive");
    for (int64_t k = 0; k < ne; ++k) c->plan.c2[k] = c2[c->plan.elem_new2old[k]];
    if (c->host_only) return SEM_OK;
    int rc = set_device(c);
    if (rc) return rc;
    SEM_HIP(c, upload_real(c, c->c2, c->plan.c2));
    if (c->geo) {
        rc = c->precision == SEM_F64 ? upload_geometry<double>(c) : upload_geometry<float>(c);
        if (rc) return rc;
    }
    // K(m) = sum_e m_e Khat_e with every Khat_e positive semi-definite and the mass
    // independent of m, so ratio * K(ref) - K(m) is positive semi-definite for
    // ratio = max_e m_e / ref_e, and lambda_max(m) <= ratio * lambda_max(ref). The power
    // iteration runs again only when that bound does not already show dt stable.
    double ratio = 0.0;
    for (int64_t k = 0; k < ne; ++k) ratio = std::max(ratio, c->plan.c2[k] / c->c2_ref[k]);
    const double bound = ratio * c->lambda_ref;
    if (c->lambda_ref > 0.0 && c->plan.dt < 2.0 / std::sqrt(bound)) {
        c->lambda_max = bound;
        c->dt_stable = 2.0 / std::sqrt(bound);
        return c->precision == SEM_F64 ? zero_state<double>(c) : zero_state<float>(c);
    }
    rc = c->precision == SEM_F64 ? power_iteration<double>(c, 60) : power_iteration<float>(c, 60);
    if (rc) return rc;
    if (!(c->plan.dt < c->dt_stable))
        return fail(c, SEM_ERR_UNSTABLE_DT, "dt exceeds the stability limit of the new model");
    return SEM_OK;
}

int sem_reset(sem_ctx* c) {
    if (!c) return SEM_ERR_INVALID_ARG;
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    return c->precision == SEM_F64 ? zero_state<double>(c) : zero_state<float>(c);
}

int sem_run(sem_ctx* c, int64_t nsteps, void* traces) {
    if (!c) return SEM_ERR_INVALID_ARG;
    if (nsteps < 0) return fail(c, SEM_ERR_INVALID_ARG, "nsteps must be >= 0");
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    return c->precision == SEM_F64 ? run_t<double>(c, nsteps, traces) : run_t<float>(c, nsteps, traces);
}

int sem_step(sem_ctx* c) { return sem_run(c, 1, nullptr); }

int sem_get_field(sem_ctx* c, int32_t which, void* dev) {
    if (!c || !dev || (which != SEM_FIELD_U && which != SEM_FIELD_V)) return SEM_ERR_INVALID_ARG;
    if (which == SEM_FIELD_V && c->formulation == SEM_FORM_HEUN)
        return fail(c, SEM_ERR_INVALID_ARG, "v is element-local in the first-order formulation");
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    const void* src = which == SEM_FIELD_U ? c->u[c->cur].p : c->v.p;
    if (c->precision == SEM_F64)
        SEM_HIP(c, sem::launch_nodes_to_original<double>((const double*)src, (double*)dev,
                                                         (const int32_t*)c->n2o_node.p, c->plan.nn, c->S, shot_major(c),
                                                         c->stream));
    else
        SEM_HIP(c, sem::launch_nodes_to_original<float>((const float*)src, (float*)dev,
                                                        (const int32_t*)c->n2o_node.p, c->plan.nn, c->S, shot_major(c),
                                                         c->stream));
    return SEM_OK;
}

int sem_set_field(sem_ctx* c, int32_t which, const void* dev) {
    if (!c || !dev || (which != SEM_FIELD_U && which != SEM_FIELD_V)) return SEM_ERR_INVALID_ARG;
    if (which == SEM_FIELD_V && c->formulation == SEM_FORM_HEUN)
        return fail(c, SEM_ERR_INVALID_ARG, "v is element-local in the first-order formulation");
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    void* dst = which == SEM_FIELD_U ? c->u[c->cur].p : c->v.p;
    c->heun_pred_valid = false;
    if (c->precision == SEM_F64)
        SEM_HIP(c, sem::launch_nodes_from_original<double>((const double*)dev, (double*)dst,
                                                           (const int32_t*)c->n2o_node.p, c->plan.nn, c->S, shot_major(c),
                                                         c->stream));
    else
        SEM_HIP(c, sem::launch_nodes_from_original<float>((const float*)dev, (float*)dst,
                                                          (const int32_t*)c->n2o_node.p, c->plan.nn, c->S, shot_major(c),
                                                         c->stream));
    return SEM_OK;
}

int sem_apply_stiffness(sem_ctx* c, const void* u_dev, void* r_dev) {
    if (!c || !u_dev || !r_dev) return SEM_ERR_INVALID_ARG;
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    return c->precision == SEM_F64 ? apply_t<double>(c, u_dev, r_dev) : apply_t<float>(c, u_dev, r_dev);
}

int sem_apply_stiffness_noalloc(sem_ctx* c, const void* u_dev, void* r_dev) {
    if (!c || !u_dev || !r_dev) return SEM_ERR_INVALID_ARG;
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    const size_t bytes = (size_t)c->plan.nn * c->S * c->wsize;
    const size_t half = (bytes + 255) & ~(size_t)255;
    if (2 * half > kScratchBytes)
        return fail(c, SEM_ERR_INVALID_ARG,
                    "n_nodes * n_shots * word size = " + std::to_string(bytes) + " bytes exceeds the " +
                        std::to_string(kScratchBytes / 2) + " bytes of one half of the scratch");
    void* base = nullptr;
    rc = scratch_address(c, &base);
    if (rc) return rc;
    void* tin = base;
    void* tout = (unsigned char*)base + half;
    return c->precision == SEM_F64 ? apply_into<double>(c, u_dev, r_dev, tin, tout)
                                   : apply_into<float>(c, u_dev, r_dev, tin, tout);
}

int sem_adjoint_gradient(sem_ctx* c, const void* dL, int64_t nsteps, int32_t ckpt_every, double* grad) {
    if (c && c->formulation == SEM_FORM_HEUN)
        return fail(c, SEM_ERR_INVALID_ARG, "no adjoint for the first-order formulation");
    if (!c || !dL || !grad) return SEM_ERR_INVALID_ARG;
    if (nsteps < 1 || ckpt_every < 1) return fail(c, SEM_ERR_INVALID_ARG, "nsteps and ckpt_every must be >= 1");
    int rc = need_device(c);
    if (rc) return rc;
    rc = set_device(c);
    if (rc) return rc;
    if (c->n_rec < 1) return fail(c, SEM_ERR_INVALID_ARG, "no receivers set");
    return c->precision == SEM_F64 ? adjoint_t<double>(c, dL, nsteps, ckpt_every, grad)
                                   : adjoint_t<float>(c, dL, nsteps, ckpt_every, grad);
}

int sem_synchronize(sem_ctx* c) {
    if (!c) return SEM_ERR_INVALID_ARG;
    if (c->host_only) return SEM_OK;
    int rc = set_device(c);
    if (rc) return rc;
    SEM_HIP(c, hipStreamSynchronize(c->stream));
    return SEM_OK;
}

int sem_hilbert_index(int64_t W, int64_t H, int64_t n, const int64_t* cx, const int64_t* cy, int64_t* out) {
    if (W < 1 || H < 1 || n < 0 || (n > 0 && (!cx || !cy || !out))) return SEM_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i) {
        if (cx[i] < 0 || cx[i] >= W || cy[i] < 0 || cy[i] >= H) return SEM_ERR_INVALID_ARG;
        out[i] = sem::hilbert_index(W, H, cx[i], cy[i]);
    }
    return SEM_OK;
}

const char* sem_last_error(const sem_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

int sem_autotune(const sem_mesh* mesh, const sem_options* base, int32_t warmup, int32_t steps,
                 sem_options* best, double* best_us, double* table, int32_t table_cap, int32_t* n_tried) {
    if (!mesh || !base || !best || !best_us || steps < 1 || warmup < 0 || table_cap < 0) {
        g_create_error = "sem_autotune: bad arguments";
        return SEM_ERR_INVALID_ARG;
    }
    if (base->device < 0) {
        g_create_error = "sem_autotune needs a device";
        return SEM_ERR_NO_DEVICE;
    }
    std::vector<sem_options> cand;
    auto vary_threads = [&](const std::vector<int>& bts, sem_options o) {
        if (o.block_threads > 0) { cand.push_back(o); return; }
        for (int bt : bts) { o.block_threads = bt; cand.push_back(o); }
    };
    const int S = base->n_shots;
    const bool tri = mesh->vertices_per_element == 3;
    if (S == 1 || tri) {
        // workgroup size x tile size (own + halo elements, in workgroup passes of
        // 64 / nodes-per-element-row elements per wave)
        const int per_wave = tri ? 64 / sem::tri_nq(base->p) : 64 / (base->p + 1);
        const std::vector<int> passes = tri ? std::vector<int>{8, 14, 20} : std::vector<int>{1, 2};
        std::vector<int> bts = {256, 512, 1024};
        if (base->block_threads > 0) bts = {base->block_threads};
        for (int bt : bts) {
            sem_options o = *base;
            o.block_threads = bt;
            if (base->tile_items > 0 || base->tile_elems > 0) { cand.push_back(o); continue; }
            for (int np : passes) { o.tile_items = np * per_wave * (bt / 64); cand.push_back(o); }
        }
    } else if (S % 64 == 0 && (base->shot_lanes == 0 || base->shot_lanes == 64)) {
        sem_options o = *base;
        if (o.lds_bytes > 0) {
            vary_threads({256, 512}, o);
        } else {
            for (int kb : {24, 32, 48, 64}) { o.lds_bytes = kb * 1024; vary_threads({256, 512}, o); }
        }
    } else {
        sem_options o = *base;
        if (o.shot_lanes > 0) {
            cand.push_back(o);
        } else {
            for (int sl = 1; sl <= 16; sl *= 2)
                if (S % sl == 0) { o.shot_lanes = sl; cand.push_back(o); }
        }
    }
    if (hipSetDevice(base->device) != hipSuccess) {
        g_create_error = "sem_autotune: hipSetDevice failed";
        return SEM_ERR_HIP;
    }
    hipStream_t st = (hipStream_t)base->stream;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        g_create_error = "sem_autotune: hipEventCreate failed";
        return SEM_ERR_HIP;
    }
    int found = -1, last_rc = SEM_OK;
    std::string last_err;
    double best_t = 0.0;
    for (size_t k = 0; k < cand.size(); ++k) {
        double us = -1.0;
        sem_ctx* c = nullptr;
        int rc = sem_create(mesh, &cand[k], &c);
        if (rc == SEM_OK) {
            rc = sem_run(c, warmup, nullptr);
            if (rc == SEM_OK && hipEventRecord(ev0, st) != hipSuccess) rc = SEM_ERR_HIP;
            if (rc == SEM_OK) rc = sem_run(c, steps, nullptr);
            if (rc == SEM_OK && hipEventRecord(ev1, st) != hipSuccess) rc = SEM_ERR_HIP;
            if (rc == SEM_OK && hipEventSynchronize(ev1) != hipSuccess) rc = SEM_ERR_HIP;
            float ms = 0.0f;
            if (rc == SEM_OK && hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) rc = SEM_ERR_HIP;
            if (rc == SEM_OK) us = 1e3 * (double)ms / steps;
            else last_err = sem_last_error(c);
            sem_destroy(c);
        } else {
            last_err = g_create_error;
        }
        if (rc != SEM_OK) last_rc = rc;
        if (us > 0.0 && (found < 0 || us < best_t)) {
            found = (int)k;
            best_t = us;
        }
        if (table && (int32_t)k < table_cap) {
            table[5 * k + 0] = cand[k].block_threads;
            table[5 * k + 1] = cand[k].shot_lanes;
            table[5 * k + 2] = cand[k].lds_bytes;
            table[5 * k + 3] = cand[k].tile_items;
            table[5 * k + 4] = us;
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (n_tried) *n_tried = (int32_t)cand.size();
    if (found < 0) {
        g_create_error = "sem_autotune: no candidate could run: " + last_err;
        return last_rc != SEM_OK ? last_rc : SEM_ERR_INVALID_ARG;
    }
    *best = cand[found];
    *best_us = best_t;
    return SEM_OK;
}

void sem_destroy(sem_ctx* c) {
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        DevBuf* bufs[] = {&c->conn, &c->G, &c->c2, &c->dtminv, &c->tile_eb, &c->tile_nb, &c->tile_ns, &c->halo_b,
                          &c->halo, &c->n2o_node, &c->n2o_elem, &c->u[0], &c->u[1], &c->v,
                          &c->src_b, &c->src_loc, &c->src_shot, &c->src_w, &c->rec_b, &c->rec_loc,
                          &c->rec_idx, &c->u_next, &c->hv[0], &c->hv[1], &c->minv_w, &c->u_pred,
                          &c->racc, &c->src_node, &c->rec_node, &c->tri_S, &c->tile_nbd,
                          &c->border_nodes, &c->brec_idx, &c->brec_node};
        for (DevBuf* b : bufs) dev_free(*b);
    }
    delete c;
}

}  // extern "C"
