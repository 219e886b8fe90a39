// kernels.hip -- gfx950 kernels of the Hilbert-ordered SEM time step.
//
// One fused launch per time step. Workgroup = one tile of consecutive elements in curve
// order x one slice of `SL` shots. The tile owns the contiguous range of global nodes its
// elements touch first (first-touch numbering makes it contiguous). The workgroup
//   1. zeroes an LDS accumulator for its owned nodes,
//   2. for every own element and every halo element (an element of another tile that
//      touches an owned node): gathers u at the element's (p+1)^2 nodes, applies the
//      tensor-product stiffness (D along each reference axis, geometric factors, D^T;
//      Eqs. deriv_u and R of the paper in second-order form) and adds the contributions
//      that land on owned nodes into LDS,
//   3. subtracts point-source terms (Alg. 3) or adjoint injections,
//   4. applies the diagonal-mass-inverse leapfrog update to its owned nodes:
//      v += dt M^-1 (f - K u), u_out = u_in + dt v,
//   5. records receivers it owns.
// Halo recomputation replaces the paper's element colouring: every contribution to a
// node is summed in its owner's LDS, so no global atomics and no second pass are needed,
// and u is double-buffered (u_in -> u_out) so tiles never read a value updated in the
// same launch.
#include <hip/hip_runtime.h>

#include "kernels.h"

// minimum waves per SIMD the register allocation must allow (FP32, FP64)
#ifndef SEM_MIN_WAVES_F32
#define SEM_MIN_WAVES_F32 3
#endif
#ifndef SEM_MIN_WAVES_F64
#define SEM_MIN_WAVES_F64 1
#endif

namespace sem {
namespace {

__device__ __forceinline__ double ricker(double t, double f0, double t0) {
    const double x = 3.14159265358979323846 * f0 * (t - t0);
    const double a = x * x;
    return (1.0 - 2.0 * a) * exp(-a);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run
// of logical block ids so that curve-neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_logical_block() {
    const int b = blockIdx.x, nblk = gridDim.x;
    const int q8 = nblk >> 3, r8 = nblk & 7, x = b & 7;
    return x * q8 + min(x, r8) + (b >> 3);
}

// Raw buffer loads: 128-bit descriptor in SGPRs, 32-bit byte offset in one VGPR, and
// reads past the descriptor's byte count return 0 instead of touching other memory.
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ int bload<int>(rsrc_t r, uint32_t off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// Raw buffer stores (vector memory), same 32-bit offsets; stores past the descriptor's
// byte count are dropped.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// N consecutive dwords with the widest loads available (16, 8, then 4 bytes)
template <int N>
__device__ __forceinline__ void load_ids(rsrc_t r, uint32_t off, int (&out)[N]) {
    int k = 0;
#pragma unroll
    for (; k + 4 <= N; k += 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off + 4u * k, 0, 0);
        out[k] = (int)v[0]; out[k + 1] = (int)v[1]; out[k + 2] = (int)v[2]; out[k + 3] = (int)v[3];
    }
    if constexpr (N % 4 >= 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off + 4u * k, 0, 0);
        out[k] = (int)v[0]; out[k + 1] = (int)v[1];
        k += 2;
    }
    if constexpr (N % 2 == 1) out[N - 1] = (int)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * (N - 1), 0, 0);
}

// one element record of 8 words (bilinear coefficients, c^2, padding) in 16-byte loads
__device__ __forceinline__ void load_rec8(rsrc_t r, uint32_t off, float (&out)[8]) {
    // lanes converted by value: __builtin_bit_cast applied to a vector-element lvalue
    // reads lane 0 for every index
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
    out[0] = __uint_as_float(v0[0]);
    out[1] = __uint_as_float(v0[1]);
    out[2] = __uint_as_float(v0[2]);
    out[3] = __uint_as_float(v0[3]);
    out[4] = __uint_as_float(v1[0]);
    out[5] = __uint_as_float(v1[1]);
    out[6] = __uint_as_float(v1[2]);
    out[7] = __uint_as_float(v1[3]);
}
__device__ __forceinline__ void load_rec8(rsrc_t r, uint32_t off, double (&out)[8]) {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off + 8u * k, 0, 0);
        out[k] = __builtin_bit_cast(double, ((unsigned long long)v[1] << 32) | v[0]);
        out[k + 1] = __builtin_bit_cast(double, ((unsigned long long)v[3] << 32) | v[2]);
    }
}

// Copy `ndw` consecutive dwords starting at byte `off` of a buffer into LDS with
// direct-to-LDS loads (no registers): each wave moves 64-dword chunks; the data lands
// asynchronously and is visible to the workgroup after s_waitcnt vmcnt(0) + barrier.
template <int RB>
__device__ __forceinline__ void lds_prefetch(rsrc_t r, uint32_t off, void* lds, int ndw) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wave; c * 64 < ndw; c += RB / 64) {
        auto* dst = (__attribute__((address_space(3))) void*)((char*)lds + c * 256);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 4, off + (uint32_t)(c * 64 + lane) * 4u, 0, 0, 0);
    }
}

// Scheduling fence: the machine scheduler may not move instructions across it, so loads
// of one stage are not hoisted into the previous one (bounds the registers live at once).
__device__ __forceinline__ void stage_fence() { __builtin_amdgcn_sched_barrier(0); }

template <int SL, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int m = 1; m < SL; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// 1/x: hardware reciprocal in FP32 (1 ulp), correctly rounded division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename T, int P, int SL>
__global__ void __launch_bounds__(kBlock, sizeof(T) == 8 ? SEM_MIN_WAVES_F64 : SEM_MIN_WAVES_F32) step_kernel(const StepArgs<T> a) {
    constexpr int N = P + 1, NQ = N * N;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* acc = reinterpret_cast<double*>(smem_raw);   // FP64 in either precision

    const int logical = xcd_logical_block();
    const int tile = logical / a.n_slices;
    const int s0 = (logical - tile * a.n_slices) * SL;
    const int nb = a.tile_nb[tile];
    const int nown = a.tile_nb[tile + 1] - nb;
    const int eb = a.tile_eb[tile];
    const int n_own_el = a.tile_eb[tile + 1] - eb;
    const int hb = a.halo_b[tile];
    const int n_halo = a.halo_b[tile + 1] - hb;
    const int S = a.S;

    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_c2 = make_rsrc(a.c2, a.c2_bytes);
    const rsrc_t r_u = make_rsrc(a.u_in, a.state_bytes);
    const rsrc_t r_pair = make_rsrc(a.u_pair, a.u_pair ? a.state_bytes : 0u);
    const uint32_t ustride = (uint32_t)S * (uint32_t)sizeof(T);

    for (int i = threadIdx.x; i < nown * SL; i += kBlock) acc[i] = 0.0;
    __syncthreads();

    const int n_items = (n_own_el + n_halo) * SL;
    for (int item = threadIdx.x; item < n_items; item += kBlock) {
        const int k = item / SL;
        const int s = item - k * SL;
        const bool own = k < n_own_el;
        const int e = own ? eb + k : a.halo[hb + k - n_own_el];
        // element-blocked layouts: [E/64][component][q][64]; one byte offset per thread
        const uint32_t eoff = (uint32_t)((e >> 6) * (NQ * 64) + (e & 63)) * 4u;
        const uint32_t goff = (uint32_t)((e >> 6) * (3 * NQ * 64) + (e & 63)) * (uint32_t)sizeof(T);
        const uint32_t soff = (uint32_t)(s0 + s) * (uint32_t)sizeof(T);
        T u[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int node = bload<int>(r_conn, eoff + q * 256);
            u[q] = bload<T>(r_u, (uint32_t)node * ustride + soff);
        }
        stage_fence();
        // Row by row (second reference index j): reference gradient at the row's GLL
        // points, geometric flux, then both D^T contractions folded in at once:
        //   r[a, j] += sum_i D[i, a] f1[i, j]   (first-axis flux of row j is complete)
        //   r[a, b] += D[j, b] f2[a, j]          (second-axis flux summed over rows)
        // so only u, r and one row of flux are live.
        T r[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) r[q] = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T f1[N], f2[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T gx = T(0), gy = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    gx += a.D[i * N + m] * u[m + N * j];
                    gy += a.D[j * N + m] * u[i + N * m];
                }
                const int q = i + N * j;
                const T g11 = bload<T>(r_G, goff + q * 64 * (uint32_t)sizeof(T));
                const T g12 = bload<T>(r_G, goff + (NQ + q) * 64 * (uint32_t)sizeof(T));
                const T g22 = bload<T>(r_G, goff + (2 * NQ + q) * 64 * (uint32_t)sizeof(T));
                f1[i] = g11 * gx + g12 * gy;
                f2[i] = g12 * gx + g22 * gy;
            }
#pragma unroll
            for (int aa = 0; aa < N; ++aa) {
                T acc1 = r[aa + N * j];
#pragma unroll
                for (int i = 0; i < N; ++i) acc1 += a.D[i * N + aa] * f1[i];
                r[aa + N * j] = acc1;
            }
#pragma unroll
            for (int bb = 0; bb < N; ++bb) {
#pragma unroll
                for (int aa = 0; aa < N; ++aa) r[aa + N * bb] += a.D[j * N + bb] * f2[aa];
            }
            stage_fence();
        }
        const T c2 = bload<T>(r_c2, (uint32_t)e * (uint32_t)sizeof(T));
        const bool pair = own && a.grad != nullptr;
        T dot = T(0);
        // scatter the owned entries into LDS. The node ids are re-read here (cache hits)
        // rather than kept live through the contraction. Element-interior nodes belong to
        // this element alone (plain store); edge and corner nodes are shared (atomics).
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int node = bload<int>(r_conn, eoff + q * 256);
            if (pair) dot += r[q] * bload<T>(r_pair, (uint32_t)node * ustride + soff);
            const int loc = node - nb;
            const int qa = q % N, qb = q / N;
            if ((unsigned)loc < (unsigned)nown) {
                if (qa > 0 && qa < P && qb > 0 && qb < P) acc[loc * SL + s] = (double)(c2 * r[q]);
                else atomicAdd(&acc[loc * SL + s], (double)(c2 * r[q]));
            }
        }
        if (a.grad != nullptr) {
            // every lane of an SL-group is active together (items are SL-aligned)
            dot = group_sum<SL>(dot);
            if (pair && s == 0) atomicAdd(&a.grad[e], (double)dot);
        }
    }
    __syncthreads();

    // point sources of this tile: acc -= w * ricker(t)
    if (a.src_b != nullptr) {
        const int sb = a.src_b[tile], se = a.src_b[tile + 1];
        if (se > sb) {
            const T amp = (T)ricker(a.src_t, a.f0, a.t0);
            for (int i = sb + threadIdx.x; i < se; i += kBlock) {
                const int sh = a.src_shot[i] - s0;
                if ((unsigned)sh < (unsigned)SL) atomicAdd(&acc[a.src_loc[i] * SL + sh], -(double)(a.src_w[i] * amp));
            }
            __syncthreads();
        }
    }
    // adjoint injection at receivers: acc -= inj[s][r][col] * scale
    if (a.inj != nullptr) {
        const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
        if (re > rb) {
            for (int i = threadIdx.x; i < (re - rb) * SL; i += kBlock) {
                const int k = rb + i / SL, s = i % SL;
                const T val = a.inj[((int64_t)(s0 + s) * a.n_rec + a.rec_idx[k]) * a.inj_cols + a.inj_col];
                atomicAdd(&acc[a.rec_loc[k] * SL + s], -(double)(val * a.inj_scale));
            }
            __syncthreads();
        }
    }

    if (a.mode == 0) {
        for (int i = threadIdx.x; i < nown * SL; i += kBlock) {
            const int loc = i / SL, s = i - (i / SL) * SL;
            const int node = nb + loc;
            const int64_t g = (int64_t)node * S + s0 + s;
            const T vn = a.v[g] - a.dtminv[node] * (T)acc[i];
            a.v[g] = vn;
            const T un = a.u_in[g] + a.dt * vn;
            a.u_out[g] = un;
            acc[i] = (double)un;
        }
        if (a.trace != nullptr) {
            const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
            if (re > rb) {
                __syncthreads();
                for (int i = threadIdx.x; i < (re - rb) * SL; i += kBlock) {
                    const int k = rb + i / SL, s = i % SL;
                    a.trace[((int64_t)(s0 + s) * a.n_rec + a.rec_idx[k]) * a.trace_cols + a.trace_col] =
                        (T)acc[a.rec_loc[k] * SL + s];
                }
            }
        }
    } else {
        for (int i = threadIdx.x; i < nown * SL; i += kBlock) {
            const int loc = i / SL, s = i - (i / SL) * SL;
            const int node = nb + loc;
            const int64_t g = (int64_t)node * S + s0 + s;
            a.r_out[g] = a.mode == 2 ? a.dtminv[node] * (T)acc[i] : (T)acc[i];
        }
    }
}

// ---------------------------------------------------------------------------------------
// Shot batches of 64: one wave per element, lane = shot. The element's node ids, its
// stored geometric factors, c^2 and the dt/M of its interior nodes are wave-uniform: they
// are read with one word per lane and broadcast with readlane. The gathers read one
// contiguous 64-shot row per node and the LDS accumulator [shared node][64 shots] is hit
// by 64 consecutive words per instruction (no bank conflicts).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)p;
}

// value of lane l (a wave-uniform constant) of v, as a scalar
template <typename T>
__device__ __forceinline__ T rlane(T v, int l);
template <>
__device__ __forceinline__ float rlane<float>(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ double rlane<double>(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// BORDER (scatter ATOMIC): tiles process their own elements only. Owned nodes whose elements
// all lie in the tile are summed in LDS as above; a border node (touched by another tile's
// elements) receives -dt/M c^2 (K_e u_e) from every element through global FP atomics on its
// 64-shot row of v (r_out in modes 1, 2), and border_update_kernel forms its u_out after the
// launch. No halo element is recomputed and no halo row gathered.
//
// GRAD: the adjoint step, which also pairs each element's K_e u with u_pair (in FP32 a
// separate instantiation, so the forward loop holds no loads that only the adjoint needs;
// FP64 runs this one for both, the pairing skipped when grad is null: without that branch
// its forward step took 218 VGPRs, two waves per SIMD instead of three).
// FP32 defers each element's interior-node stores until the next element's loads are issued:
// a wave's loads and stores complete in issue order, so stores issued before a load would be
// waited for together with it.
template <typename T, int P, int BT, bool BORDER, bool GRAD>
__global__ void __launch_bounds__(BT)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && P <= 4 ? 4 : 1, 8)))
    step_shots_kernel(const StepArgs<T> a) {
    constexpr int N = P + 1, NQ = N * N, SL = 64, NW = BT / 64;
    constexpr int NI = (P - 1) * (P - 1);              // element-interior nodes
    constexpr int REC = 3 * NQ + 1 + NI;               // g11[nq] g12[nq] g22[nq] c2 dt/M[ni]
    constexpr int NREG = (REC + 63) / 64;
    constexpr int U = 4;                               // nodes per wave per update round
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // [shared owned][64] in FP64 for either precision: ds_add_f64 sustains a much higher
    // rate than ds_add_f32 here (the FP32 step ran 1.3x faster with FP64 accumulators),
    // and the sum rounds once
    double* acc = reinterpret_cast<double*>(smem_raw);

    const int logical = xcd_logical_block();
    const int tile = logical / a.n_slices;
    const int s0 = (logical - tile * a.n_slices) * SL;
    const int nb = a.tile_nb[tile];
    const int nown = a.tile_nb[tile + 1] - nb;
    const int ns = a.tile_ns[tile];                     // owned nodes on an element edge (BORDER:
                                                        // whose elements all lie in this tile)
    const int nbd = BORDER ? a.tile_nbd[tile] : 0;     // BORDER: owned border nodes, after those
    const int eb = a.tile_eb[tile];
    const int n_own_el = a.tile_eb[tile + 1] - eb;
    const int hb = a.halo_b[tile];
    const int n_items = n_own_el + (BORDER ? 0 : a.halo_b[tile + 1] - hb);
    const int S = a.S;
    const cptr<int32_t> halo = as_const(a.halo);
    const cptr<T> dtminv = as_const(a.dtminv);
    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_u = make_rsrc(a.u_in, a.state_bytes);
    const rsrc_t r_v = make_rsrc(a.v, a.state_bytes);
    const rsrc_t r_uo = make_rsrc(a.u_out, a.u_out ? a.state_bytes : 0u);
    const rsrc_t r_ro = make_rsrc(a.r_out, a.r_out ? a.state_bytes : 0u);
    const rsrc_t r_pair = make_rsrc(a.u_pair, a.u_pair ? a.state_bytes : 0u);
    const uint32_t ustride = (uint32_t)S * (uint32_t)sizeof(T);
    // this tile's point sources and receivers (per-tile lists, usually empty)
    const int sb = a.src_b ? a.src_b[tile] : 0, se = a.src_b ? a.src_b[tile + 1] : 0;
    const int rb = a.rec_b ? a.rec_b[tile] : 0, re = a.rec_b ? a.rec_b[tile + 1] : 0;
    const T amp = se > sb ? (T)ricker(a.src_t, a.f0, a.t0) : T(0);

    for (int i = threadIdx.x; i < ns * SL; i += BT) acc[i] = 0.0;
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t soff = (uint32_t)(s0 + lane) * (uint32_t)sizeof(T);
    // element k of the tile: own elements first, then the halo
    auto elem_of = [&](int k) { return k < n_own_el ? eb + k : halo[hb + k - n_own_el]; };
    // An element's node ids (lane q holds id q) and its record (word i in lane i % 64 of
    // register i / 64) are read one element ahead, into VGPRs, and broadcast with readlane.
    // The loads in the element loop are unconditional (past the last element, or where a value
    // is not needed, a lane reads at the buffer's byte count, which returns 0), so the waits
    // count exactly what they need.
    auto load_ids = [&](bool act, int e) {
        return bload<int>(r_conn, act ? (uint32_t)(e * NQ + (lane < NQ ? lane : 0)) * 4u : a.conn_bytes);
    };
    auto load_rec = [&](bool act, int e, T* gv) {
#pragma unroll
        for (int rg = 0; rg < NREG; ++rg) {
            const int w = rg * 64 + lane;
            gv[rg] = bload<T>(r_G, act ? (uint32_t)(e * REC + (w < REC ? w : 0)) * (uint32_t)sizeof(T) : a.G_bytes);
        }
    };
    constexpr bool DEFER = sizeof(T) == 4;
    constexpr int ND = DEFER && NI > 0 ? NI : 1;
    // the element-interior results of the previous element (mode 0: v and u_out; modes 1, 2:
    // r_out) and that element's ids; st_d: whether it is an own element
    T dv0[ND], dv1[ND];
    int cv_d = 0;
    bool st_d = false;
    const bool mode0 = a.mode == 0;
    const rsrc_t r_s0 = mode0 ? r_v : r_ro, r_s1 = mode0 ? r_uo : r_ro;
    auto flush = [&]() {
#pragma unroll
        for (int b = 1; b < P; ++b)
#pragma unroll
            for (int c = 1; c < P; ++c) {
                const int ii = (b - 1) * (P - 1) + c - 1;
                const uint32_t off = st_d ? (uint32_t)__builtin_amdgcn_readlane(cv_d, c + N * b) * ustride + soff
                                          : a.state_bytes;
                bstore(r_s0, off, dv0[ii]);
                bstore(r_s1, mode0 ? off : a.state_bytes, dv1[ii]);
            }
    };
    const bool act0 = wave < n_items;
    int e_next = act0 ? elem_of(wave) : 0;
    int cv_next = load_ids(act0, e_next);
    T gv_next[NREG];
    load_rec(act0, e_next, gv_next);
    for (int k = wave; k < n_items; k += NW) {
        const bool own = k < n_own_el;
        const int e = e_next;
        const int cv = cv_next;
        T gv[NREG];
#pragma unroll
        for (int rg = 0; rg < NREG; ++rg) gv[rg] = gv_next[rg];
        T u[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            u[q] = bload<T>(r_u, (uint32_t)__builtin_amdgcn_readlane(cv, q) * ustride + soff);
        // v at the element-interior nodes (nodes of this element alone, finished below):
        // requested now so that the loads overlap the contraction
        const bool upd = own && mode0;
        T vin[NI > 0 ? NI : 1];
        // FP64 (no deferred stores, so no exact wait to keep) issues these loads only where
        // they are needed
        if (DEFER || upd) {
#pragma unroll
            for (int b = 1; b < P; ++b)
#pragma unroll
                for (int c = 1; c < P; ++c)
                    vin[(b - 1) * (P - 1) + c - 1] =
                        bload<T>(r_v, upd ? (uint32_t)__builtin_amdgcn_readlane(cv, c + N * b) * ustride + soff
                                          : a.state_bytes);
        }
        const bool act_n = k + NW < n_items;
        if (DEFER || act_n) {
            e_next = act_n ? elem_of(k + NW) : 0;
            cv_next = load_ids(act_n, e_next);
            load_rec(act_n, e_next, gv_next);
        }
        if constexpr (DEFER) flush();
        // word w of the record
        auto rec = [&](int w) { return rlane(gv[w / 64], w % 64); };
        T r[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) r[q] = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T f1[N], f2[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T gx = T(0), gy = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    gx += a.D[i * N + m] * u[m + N * j];
                    gy += a.D[j * N + m] * u[i + N * m];
                }
                const int q = i + N * j;
                const T g11 = rec(q), g12 = rec(NQ + q), g22 = rec(2 * NQ + q);
                f1[i] = g11 * gx + g12 * gy;
                f2[i] = g12 * gx + g22 * gy;
            }
#pragma unroll
            for (int aa = 0; aa < N; ++aa) {
                T s1 = r[aa + N * j];
#pragma unroll
                for (int i = 0; i < N; ++i) s1 += a.D[i * N + aa] * f1[i];
                r[aa + N * j] = s1;
            }
#pragma unroll
            for (int bb = 0; bb < N; ++bb) {
#pragma unroll
                for (int aa = 0; aa < N; ++aa) r[aa + N * bb] += a.D[j * N + bb] * f2[aa];
            }
        }
        const T c2 = rec(3 * NQ);
        if constexpr (GRAD) {
            if (a.grad != nullptr && own) {
                T dot = T(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    dot += r[q] * bload<T>(r_pair, (uint32_t)__builtin_amdgcn_readlane(cv, q) * ustride + soff);
                dot = group_sum<64>(dot);
                if (lane == 0) atomicAdd(&a.grad[e], (double)dot);
            }
        }
        // Node ids are wave-uniform, so these branches do not diverge. Every owned node on an
        // element edge accumulates in LDS (BORDER: unless another tile's elements touch it);
        // an edge node owned by another tile is that tile's (a halo element's contribution).
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int qa = q % N, qb = q / N;
            if (qa > 0 && qa < P && qb > 0 && qb < P) continue;     // interior: below
            const int node = __builtin_amdgcn_readlane(cv, q);
            const int loc = node - nb;
            if ((unsigned)loc < (unsigned)ns) {
                atomicAdd(&acc[loc * SL + lane], (double)(c2 * r[q]));
            } else if (BORDER && ((unsigned)(loc - ns) < (unsigned)nbd || (unsigned)loc >= (unsigned)nown)) {
                // a border node, this tile's or another's: its sum completes after every tile
                const T rt = c2 * r[q];
                const int64_t g = (int64_t)node * S + s0 + lane;
                if (mode0) atomicAdd(&a.v[g], -(dtminv[node] * rt));
                else atomicAdd(&a.r_out[g], a.mode == 2 ? dtminv[node] * rt : rt);
            }
        }
        // element-interior nodes: single-element, owned by this element's tile
#pragma unroll
        for (int b = 1; b < P; ++b)
#pragma unroll
            for (int c = 1; c < P; ++c) {
                const int q = c + N * b, ii = (b - 1) * (P - 1) + c - 1;
                if constexpr (DEFER) {
                    const T rt = c2 * r[q];
                    const T dm = rec(3 * NQ + 1 + ii);
                    dv0[ii] = mode0 ? vin[ii] - dm * rt : (a.mode == 2 ? dm * rt : rt);
                    dv1[ii] = u[q] + a.dt * dv0[ii];
                } else if (own) {
                    const T rt = c2 * r[q];
                    const T dm = rec(3 * NQ + 1 + ii);
                    const uint32_t off = (uint32_t)__builtin_amdgcn_readlane(cv, q) * ustride + soff;
                    if (mode0) {
                        const T vn = vin[ii] - dm * rt;
                        bstore(r_v, off, vn);
                        bstore(r_uo, off, u[q] + a.dt * vn);
                    } else {
                        bstore(r_ro, off, a.mode == 2 ? dm * rt : rt);
                    }
                }
            }
        if constexpr (DEFER) {
            cv_d = cv;
            st_d = own;
        }
    }
    if constexpr (DEFER) flush();
    __syncthreads();

    // Sources and adjoint injection: force f enters as acc -= f at accumulated nodes; at
    // single-element nodes (already advanced without it) as v += dt/M f, u += dt dt/M f,
    // with global atomics (several receivers may sit on one node).
    if (se > sb) {
        for (int i = sb + threadIdx.x; i < se; i += BT) {
            const int sh = a.src_shot[i] - s0, loc = a.src_loc[i];
            if ((unsigned)sh >= (unsigned)SL) continue;
            const T f = a.src_w[i] * amp;
            if (loc < ns) {
                atomicAdd(&acc[loc * SL + sh], -(double)f);
            } else if (BORDER && loc < ns + nbd) {
                atomicAdd(&a.v[(int64_t)(nb + loc) * S + s0 + sh], a.dtminv[nb + loc] * f);
            } else {
                const int64_t g = (int64_t)(nb + loc) * S + s0 + sh;
                const T dv = a.dtminv[nb + loc] * f;
                atomicAdd(&a.v[g], dv);
                atomicAdd(&a.u_out[g], a.dt * dv);
            }
        }
        __syncthreads();
    }
    if (a.inj != nullptr && re > rb) {
        for (int i = threadIdx.x; i < (re - rb) * SL; i += BT) {
            const int kk = rb + i / SL, sh = i % SL, loc = a.rec_loc[kk];
            const T f = a.inj[((int64_t)(s0 + sh) * a.n_rec + a.rec_idx[kk]) * a.inj_cols + a.inj_col] *
                        a.inj_scale;
            if (loc < ns) {
                atomicAdd(&acc[loc * SL + sh], -(double)f);
            } else if (BORDER && loc < ns + nbd) {
                atomicAdd(&a.v[(int64_t)(nb + loc) * S + s0 + sh], a.dtminv[nb + loc] * f);
            } else {
                const int64_t g = (int64_t)(nb + loc) * S + s0 + sh;
                const T dv = a.dtminv[nb + loc] * f;
                atomicAdd(&a.v[g], dv);
                atomicAdd(&a.u_out[g], a.dt * dv);
            }
        }
        __syncthreads();
    }
    if (a.mode == 0) {
        // one wave per accumulated node, U nodes per round with all loads issued first
        for (int l0 = wave; l0 < ns; l0 += NW * U) {
            T vv[U], uu[U], mm[U], ac[U];           // ac: the accumulated K u - f, rounded
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int loc = l0 + t * NW;
                const uint32_t off = (uint32_t)(nb + loc) * ustride + soff;
                vv[t] = bload<T>(r_v, off);
                uu[t] = bload<T>(r_u, off);
                mm[t] = loc < ns ? dtminv[nb + loc] : T(0);
                ac[t] = loc < ns ? (T)acc[loc * SL + lane] : T(0);
            }
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int loc = l0 + t * NW;
                if (loc < ns) {
                    const uint32_t off = (uint32_t)(nb + loc) * ustride + soff;
                    const T vn = vv[t] - mm[t] * ac[t];
                    bstore(r_v, off, vn);
                    const T un = uu[t] + a.dt * vn;
                    bstore(r_uo, off, un);
                    acc[loc * SL + lane] = (double)un;
                }
            }
        }
        if (a.trace != nullptr && re > rb) {
            __syncthreads();
            for (int i = threadIdx.x; i < (re - rb) * SL; i += BT) {
                const int kk = rb + i / SL, sh = i % SL, loc = a.rec_loc[kk];
                if (BORDER && loc >= ns && loc < ns + nbd) continue;    // recorded after the border pass
                // single-element nodes: read back from L2 (the corrections above are atomics)
                a.trace[((int64_t)(s0 + sh) * a.n_rec + a.rec_idx[kk]) * a.trace_cols + a.trace_col] =
                    loc < ns ? (T)acc[loc * SL + sh]
                             : __hip_atomic_load(&a.u_out[(int64_t)(nb + loc) * S + s0 + sh], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
        for (int loc = wave; loc < ns; loc += NW)
            bstore(r_ro, (uint32_t)(nb + loc) * ustride + soff,
                   a.mode == 2 ? dtminv[nb + loc] * (T)acc[loc * SL + lane] : (T)acc[loc * SL + lane]);
    }
}

// ---------------------------------------------------------------------------------------
// Single-shot step, one thread per element row. p+1 consecutive lanes of a wave hold the
// p+1 rows (second reference index j) of one element; a wave holds 64/(p+1) elements and
// a 1024-thread workgroup 16 times that. The two contractions that run across rows (the
// derivative along the second axis and its D^T) exchange one element's values through a
// per-element LDS stage written and read by the same wave (LDS executes one wave's
// instructions in order, so no barrier is needed). Geometric factors come from the six
// bilinear-map coefficients of the element.
// Row-lane layout (single shot): p+1 consecutive lanes of a wave hold the p+1 rows (second
// reference index j) of one element, and the element's LDS stage `st` [nq] is written and read
// by those lanes only. A wave barrier orders every stage exchange: it keeps the compiler from
// moving LDS accesses across it, and the lanes of one wave execute LDS instructions in order.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Workgroup barrier that orders LDS only. __syncthreads() also waits for every global
// load the wave has in flight, which would hold each wave at the block's first barrier
// until the direct-to-LDS prefetch of the update operands had landed; those loads are
// waited for after the element loop instead.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);                // lgkmcnt(0): this wave's LDS writes done
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Row j of D, column j of D, xi_j and w_j in registers, selected from the uniform kernel
// arguments (no per-lane memory reads).
template <typename T, int P, typename Args>
__device__ __forceinline__ void row_constants(const Args& a, int j, T (&Dj)[P + 1], T (&DjT)[P + 1], T& xij,
                                              T& wj) {
    constexpr int N = P + 1;
    xij = a.xi[0];
    wj = a.w[0];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        Dj[m] = a.D[m];
        DjT[m] = a.D[m * N];
    }
#pragma unroll
    for (int jj = 1; jj < N; ++jj) {
        if (j == jj) {
#pragma unroll
            for (int m = 0; m < N; ++m) {
                Dj[m] = a.D[jj * N + m];
                DjT[m] = a.D[m * N + jj];
            }
            xij = a.xi[jj];
            wj = a.w[jj];
        }
    }
}

// Stiffness apply of row j of one element (Eqs. deriv_u and R, second-order flux, without
// c^2), as used by the global-accumulator kernel. step_rows_kernel carries the same
// contraction written out in its own body: its FP32 allocation is tuned to 64 VGPRs, and the
// scheduler spills inside the element loop when the code is arranged differently.
// From u[i] = u(xi_i, xi_j) and the element's bilinear-map coefficients bl[0..5]
// (x_xi = bl0 + bl2 eta, x_eta = bl1 + bl2 xi, y likewise with bl3..5), r[a] = (Khat_e u)(a, j).
// The reference gradient along the row comes from u, across rows from the stage; the
// geometric factors w_i w_j detJ J^-1 J^-T are formed at each point; D^T along the row stays
// in registers, across rows it goes through the stage again.
template <typename T, int P, typename Args>
__device__ __forceinline__ void row_stiffness(const Args& a, const T (&u)[P + 1], const T* bl, T* st, int j,
                                              const T (&Dj)[P + 1], const T (&DjT)[P + 1], T xij, T wj,
                                              T (&r)[P + 1]) {
    constexpr int N = P + 1;
#pragma unroll
    for (int i = 0; i < N; ++i) st[i + N * j] = u[i];
    wave_sync();
    T gx[N], gy[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T sacc = T(0);
#pragma unroll
        for (int m = 0; m < N; ++m) sacc += a.D[i * N + m] * u[m];
        gx[i] = sacc;
        gy[i] = T(0);
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const T djm = Dj[m];
#pragma unroll
        for (int i = 0; i < N; ++i) gy[i] += djm * st[i + N * m];
    }
    // geometric flux at (xi_i, xi_j); first-axis D^T stays in the row
    const T xs = bl[0] + bl[2] * xij;
    const T ys = bl[3] + bl[5] * xij;
    T f2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const T xt = bl[1] + bl[2] * a.xi[i];
        const T yt = bl[4] + bl[5] * a.xi[i];
        const T sc = (a.w[i] * wj) * recip(xs * yt - xt * ys);
        const T g11 = sc * (xt * xt + yt * yt);
        const T g12 = -sc * (xs * xt + ys * yt);
        const T g22 = sc * (xs * xs + ys * ys);
        const T f1 = g11 * gx[i] + g12 * gy[i];
        f2[i] = g12 * gx[i] + g22 * gy[i];
        gx[i] = f1;
    }
#pragma unroll
    for (int aa = 0; aa < N; ++aa) {
        T sacc = T(0);
#pragma unroll
        for (int i = 0; i < N; ++i) sacc += a.D[i * N + aa] * gx[i];
        r[aa] = sacc;
    }
    // second-axis D^T across rows: r[a, j] += sum_m D[m, j] f2[a, m]
    wave_sync();                                       // every lane has read the u rows
#pragma unroll
    for (int i = 0; i < N; ++i) st[i + N * j] = f2[i];
    wave_sync();
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const T dmj = DjT[m];
#pragma unroll
        for (int aa = 0; aa < N; ++aa) r[aa] += dmj * st[aa + N * m];
    }
    wave_sync();                                       // before the stage is written again
}

template <typename T, int P, int NP>
constexpr int rows_waves() {
    // FP32 p <= 4: eight waves (64 VGPRs); p >= 5 is faster left to the compiler (the graded
    // p = 5 step ran 13% faster without the 64-register cap than squeezed into it with spills)
    return sizeof(T) == 4 ? (NP == 1 ? (P <= 4 ? 8 : 1) : (NP == 2 ? 5 : 3)) : (NP == 1 ? 4 : (NP == 2 ? 3 : 2));
}

// GRAD: the adjoint step, which also pairs each element's K_e u with u_pair, reduces the
// pairing over the element's p+1 row lanes and adds it with one atomic (a separate
// instantiation, so the forward step keeps its register allocation). Several shots run
// as one launch per shot, with the state vectors ([S][N], shot-major) offset by the host.
template <typename T, int P, int RB, int NP, bool GRAD>
__global__ void __attribute__((amdgpu_flat_work_group_size(RB, RB),
                               amdgpu_waves_per_eu(GRAD ? 1 : rows_waves<T, P, NP>(), 8)))
step_rows_kernel(const StepArgs<T> a) {
    constexpr int kRowBlock = RB;                      // threads of this workgroup
    constexpr int N = P + 1, NQ = N * N;
    constexpr int NQP = (NQ + 3) & ~3;                 // 16-byte aligned stage stride
    constexpr int EPW = 64 / N;                        // elements per wave
    constexpr int EPB = EPW * (kRowBlock / 64);        // elements per workgroup pass
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* stage = reinterpret_cast<T*>(smem_raw);          // [EPB][NQP]
    // [owned nodes] in FP64 for either precision (ds_add_f64 sustains a higher rate than
    // ds_add_f32 on this chip, and the sum rounds once)
    double* acc = reinterpret_cast<double*>(stage + EPB * NQP);
    // owned v, u_in and dt/M prefetched for the update phase: [3][a.lds_own] (64-aligned)
    T* pre_v = reinterpret_cast<T*>(acc + a.lds_own);
    T* pre_u = pre_v + a.lds_own;
    T* pre_m = pre_u + a.lds_own;

    const int logical = xcd_logical_block();
    const int tile = logical;
    const int nb = a.tile_nb[tile];
    const int nown = a.tile_nb[tile + 1] - nb;
    const int eb = a.tile_eb[tile];
    const int n_own_el = a.tile_eb[tile + 1] - eb;
    const int hb = a.halo_b[tile];
    const int n_items = n_own_el + (a.halo_b[tile + 1] - hb);

    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_u = make_rsrc(a.u_in, a.state_bytes);
    const rsrc_t r_pair = make_rsrc(a.u_pair, a.u_pair ? a.state_bytes : 0u);

    if (a.mode == 0) {
        // the update phase's operands travel while the elements are processed
        const int ndw = nown * (int)(sizeof(T) / 4);
        const uint32_t off = (uint32_t)nb * (uint32_t)sizeof(T);
        lds_prefetch<RB>(make_rsrc(a.v, a.state_bytes), off, pre_v, ndw);
        lds_prefetch<RB>(r_u, off, pre_u, ndw);
        lds_prefetch<RB>(make_rsrc(a.dtminv, a.state_bytes), off, pre_m, ndw);
    }
    for (int i = threadIdx.x; i < nown; i += kRowBlock) acc[i] = 0.0;
    lds_barrier();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kw = lane / N;                           // element slot inside the wave
    const int j = lane - kw * N;                       // row of that element
    const int slot = wave * EPW + kw;
    T* st = stage + slot * NQP;
    // The row j of a thread never changes: keep row j and column j of D, xi_j and w_j in
    // registers (selected from the uniform kernel arguments, no per-lane memory reads).
    T Dj[N], DjT[N], xij = a.xi[0], wj = a.w[0];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        Dj[m] = a.D[m];
        DjT[m] = a.D[m * N];
    }
#pragma unroll
    for (int jj = 1; jj < N; ++jj) {
        if (j == jj) {
#pragma unroll
            for (int m = 0; m < N; ++m) {
                Dj[m] = a.D[jj * N + m];
                DjT[m] = a.D[m * N + jj];
            }
            xij = a.xi[jj];
            wj = a.w[jj];
        }
    }
    // NP passes at a time: every pass's indices and geometry are requested first, then
    // every pass's gathers, so a tile costs two memory round trips instead of 2 NP.
    for (int base = 0; base < n_items; base += NP * EPB) {
        int es[NP], idx[NP][N];
        bool act[NP];
        T bl[NP][8], u[NP][N];
        T dots[GRAD ? NP : 1];                         // adjoint: pairing of this row
        if constexpr (GRAD) {
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) dots[pp] = T(0);
        }
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int k = base + pp * EPB + slot;
            act[pp] = kw < EPW && k < n_items;
            es[pp] = 0;
            if (act[pp]) {
                const int e = k < n_own_el ? eb + k : a.halo[hb + k - n_own_el];
                es[pp] = e;
                // element-major records: row j's node ids, then the element's geometry + c^2
                load_ids<N>(r_conn, (uint32_t)(e * NQ + N * j) * 4u, idx[pp]);
                load_rec8(r_G, (uint32_t)e * 8u * (uint32_t)sizeof(T), bl[pp]);
            }
        }
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            if (act[pp]) {
#pragma unroll
                for (int i = 0; i < N; ++i) u[pp][i] = bload<T>(r_u, (uint32_t)idx[pp][i] * (uint32_t)sizeof(T));
            }
        }
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            if (!act[pp]) continue;
            const int k = base + pp * EPB + slot;
            const bool own = k < n_own_el;
            const int e = es[pp];
#pragma unroll
            for (int i = 0; i < N; ++i) st[i + N * j] = u[pp][i];
            wave_sync();
            // reference gradient at the row's points: d/dxi from the row, d/deta from the stage
            T gx[N], gy[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T sacc = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) sacc += a.D[i * N + m] * u[pp][m];
                gx[i] = sacc;
                gy[i] = T(0);
            }
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const T djm = Dj[m];
#pragma unroll
                for (int i = 0; i < N; ++i) gy[i] += djm * st[i + N * m];
            }
            // geometric flux at (xi_i, xi_j); first-axis D^T stays in the row
            const T xs = bl[pp][0] + bl[pp][2] * xij;
            const T ys = bl[pp][3] + bl[pp][5] * xij;
            T f2[N], r[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T xt = bl[pp][1] + bl[pp][2] * a.xi[i];
                const T yt = bl[pp][4] + bl[pp][5] * a.xi[i];
                const T sc = (a.w[i] * wj) * recip(xs * yt - xt * ys);
                const T g11 = sc * (xt * xt + yt * yt);
                const T g12 = -sc * (xs * xt + ys * yt);
                const T g22 = sc * (xs * xs + ys * ys);
                const T f1 = g11 * gx[i] + g12 * gy[i];
                f2[i] = g12 * gx[i] + g22 * gy[i];
                gx[i] = f1;
            }
#pragma unroll
            for (int aa = 0; aa < N; ++aa) {
                T sacc = T(0);
#pragma unroll
                for (int i = 0; i < N; ++i) sacc += a.D[i * N + aa] * gx[i];
                r[aa] = sacc;
            }
            // second-axis D^T across rows: r[a, j] += sum_m D[m, j] f2[a, m]
            wave_sync();                               // every lane has read the u rows
#pragma unroll
            for (int i = 0; i < N; ++i) st[i + N * j] = f2[i];
            wave_sync();
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const T dmj = DjT[m];
#pragma unroll
                for (int aa = 0; aa < N; ++aa) r[aa] += dmj * st[aa + N * m];
            }
            wave_sync();                               // before the stage is written again
            if constexpr (GRAD) {
                if (own) {
                    T dot = T(0);
#pragma unroll
                    for (int aa = 0; aa < N; ++aa)
                        dot += r[aa] * bload<T>(r_pair, (uint32_t)idx[pp][aa] * (uint32_t)sizeof(T));
                    dots[pp] = dot;
                }
            } else if (a.grad != nullptr && own) {
                // Not reached: forward launches carry no gradient. It stays because the
                // scheduler then keeps the tuned allocation of the FP32 p = 4 step (64 VGPRs,
                // 1 spilled); without it 13 VGPRs spill inside the element loop and the step
                // ran 38% slower on the layered 1024^2 mesh.
                T dot = T(0);
#pragma unroll
                for (int aa = 0; aa < N; ++aa)
                    dot += r[aa] * bload<T>(r_pair, (uint32_t)idx[pp][aa] * (uint32_t)sizeof(T));
                atomicAdd(&a.grad[e], (double)dot);
            }
            // Element-interior nodes (0 < a, j < p) belong to this element alone: a plain
            // LDS store; nodes on element edges and corners are shared and need atomics.
            const bool inner_row = j > 0 && j < P;
#pragma unroll
            for (int aa = 0; aa < N; ++aa) {
                const int loc = idx[pp][aa] - nb;
                if ((unsigned)loc < (unsigned)nown) {
                    if (aa > 0 && aa < P && inner_row) acc[loc] = (double)(bl[pp][6] * r[aa]);
                    else atomicAdd(&acc[loc], (double)(bl[pp][6] * r[aa]));
                }
            }
        }
        if constexpr (GRAD) {
            // all lanes active again: sum the N rows of each element, one atomic per element
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) {
                T tot = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) tot += __shfl(dots[pp], kw * N + m, 64);
                if (j == 0 && act[pp] && base + pp * EPB + slot < n_own_el)
                    atomicAdd(&a.grad[es[pp]], (double)tot);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);                     // this wave's LDS prefetches landed
    __syncthreads();

    if (a.src_b != nullptr) {
        const int sb = a.src_b[tile], se = a.src_b[tile + 1];
        if (se > sb) {
            const T amp = (T)ricker(a.src_t, a.f0, a.t0);
            for (int i = sb + threadIdx.x; i < se; i += kRowBlock)
                if (a.src_shot[i] == a.shot) atomicAdd(&acc[a.src_loc[i]], -(double)(a.src_w[i] * amp));
            __syncthreads();
        }
    }
    if (a.inj != nullptr) {
        const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
        if (re > rb) {
            for (int i = rb + threadIdx.x; i < re; i += kRowBlock) {
                const T val = a.inj[(int64_t)a.rec_idx[i] * a.inj_cols + a.inj_col];
                atomicAdd(&acc[a.rec_loc[i]], -(double)(val * a.inj_scale));
            }
            __syncthreads();
        }
    }
    if (a.mode == 0) {
        // owned-node update from the prefetched operands
        for (int i = threadIdx.x; i < nown; i += kRowBlock) {
            const T vn = pre_v[i] - pre_m[i] * (T)acc[i];
            const T un = pre_u[i] + a.dt * vn;
            a.v[nb + i] = vn;
            a.u_out[nb + i] = un;
            acc[i] = (double)un;
        }
        if (a.trace != nullptr) {
            const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
            if (re > rb) {
                __syncthreads();
                for (int i = rb + threadIdx.x; i < re; i += kRowBlock)
                    a.trace[(int64_t)a.rec_idx[i] * a.trace_cols + a.trace_col] = (T)acc[a.rec_loc[i]];
            }
        }
    } else {
        for (int i = threadIdx.x; i < nown; i += kRowBlock)
            a.r_out[nb + i] = a.mode == 2 ? a.dtminv[nb + i] * (T)acc[i] : (T)acc[i];
    }
}

// ---------------------------------------------------------------------------------------
// Global accumulator (SEM_SCATTER_COLOUR and SEM_SCATTER_ATOMIC): the paper's structure of a
// step (Alg. 2 then the update): every element adds its contribution into a global r, then a
// node pass applies the update. Single shot, row-lane layout of step_rows_kernel, one
// workgroup per 64 / (p+1) * RB / 64 consecutive elements of the launch range, XCD-aware.
template <typename T, int P, int RB, bool ATOMIC, bool GRAD>
__global__ void __attribute__((amdgpu_flat_work_group_size(RB, RB))) elem_rows_kernel(const StepArgs<T> a) {
    constexpr int N = P + 1, NQ = N * N;
    constexpr int NQP = (NQ + 3) & ~3;
    constexpr int EPW = 64 / N;
    constexpr int EPB = EPW * (RB / 64);
    __shared__ __align__(16) T stage[EPB * NQP];
    const int blk = xcd_logical_block();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kw = lane / N, j = lane - kw * N;
    const int slot = wave * EPW + kw;
    const int k = blk * EPB + slot;
    // all p+1 lanes of an element leave together, so the stage exchange stays intact
    if (kw >= EPW || k >= a.e_count) return;
    const int e = a.e_begin + k;
    T* st = stage + slot * NQP;
    T Dj[N], DjT[N], xij, wj;
    row_constants<T, P>(a, j, Dj, DjT, xij, wj);
    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_u = make_rsrc(a.u_in, a.state_bytes);
    int idx[N];
    load_ids<N>(r_conn, (uint32_t)(e * NQ + N * j) * 4u, idx);
    T bl[8];
    load_rec8(r_G, (uint32_t)e * 8u * (uint32_t)sizeof(T), bl);
    T u[N];
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = bload<T>(r_u, (uint32_t)idx[i] * (uint32_t)sizeof(T));
    T r[N];
    row_stiffness<T, P>(a, u, bl, st, j, Dj, DjT, xij, wj, r);
    if constexpr (GRAD) {
        const rsrc_t r_pair = make_rsrc(a.u_pair, a.state_bytes);
        T dot = T(0);
#pragma unroll
        for (int aa = 0; aa < N; ++aa) dot += r[aa] * bload<T>(r_pair, (uint32_t)idx[aa] * (uint32_t)sizeof(T));
        T tot = T(0);
#pragma unroll
        for (int m = 0; m < N; ++m) tot += __shfl(dot, kw * N + m, 64);
        if (j == 0) atomicAdd(&a.grad[e], (double)tot);
    }
    // element-interior nodes (0 < a, j < p) belong to this element alone: plain stores
    const bool inner_row = j > 0 && j < P;
#pragma unroll
    for (int aa = 0; aa < N; ++aa) {
        const T val = bl[6] * r[aa];
        T* dst = a.racc + idx[aa];
        if (aa > 0 && aa < P && inner_row) *dst = val;
        else if constexpr (ATOMIC) atomicAdd(dst, val);
        else *dst += val;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) node_update_kernel(const StepArgs<T> a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T r = a.racc[i];
        a.racc[i] = T(0);
        if (a.mode == 0) {
            const T vn = a.v[i] - a.dtminv[i] * r;
            a.v[i] = vn;
            a.u_out[i] = a.u_in[i] + a.dt * vn;
        } else {
            a.r_out[i] = a.mode == 2 ? a.dtminv[i] * r : r;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) global_points_kernel(const StepArgs<T> a, int phase) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (phase == 0) {
        if (a.src_node != nullptr && i < a.n_src_pts && a.src_shot[i] == a.shot)
            atomicAdd(&a.racc[a.src_node[i]], -(a.src_w[i] * (T)ricker(a.src_t, a.f0, a.t0)));
        if (a.inj != nullptr && i < a.n_rec_pts)
            atomicAdd(&a.racc[a.rec_node[i]],
                      -(a.inj[(int64_t)a.rec_idx[i] * a.inj_cols + a.inj_col] * a.inj_scale));
    } else if (a.trace != nullptr && i < a.n_rec_pts) {
        a.trace[(int64_t)a.rec_idx[i] * a.trace_cols + a.trace_col] = a.u_out[a.rec_node[i]];
    }
}

template <typename T, int P, int RB>
hipError_t launch_elems_p(bool atomic, const StepArgs<T>& a, hipStream_t st) {
    constexpr int EPB = (64 / (P + 1)) * (RB / 64);
    if (a.e_count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.e_count + EPB - 1) / EPB);
    auto fn = atomic ? (a.grad ? elem_rows_kernel<T, P, RB, true, true> : elem_rows_kernel<T, P, RB, true, false>)
                     : (a.grad ? elem_rows_kernel<T, P, RB, false, true> : elem_rows_kernel<T, P, RB, false, false>);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(RB), 0, st, a);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_elems_t(int threads, bool atomic, const StepArgs<T>& a, hipStream_t st) {
    switch (threads) {
        case 256: return launch_elems_p<T, P, 256>(atomic, a, st);
        case 512: return launch_elems_p<T, P, 512>(atomic, a, st);
        case 1024: return launch_elems_p<T, P, 1024>(atomic, a, st);
        default: return hipErrorInvalidValue;
    }
}

// Vertex rotations of the triangle's local node numbering (node (i, j) at index
// j (P + 1) - j (j - 1) / 2 + i, k = P - i - j): s23 takes node (i, j, k) to (j, k, i), s13 to
// (k, i, j), s13 = s23^-1. The host checks that they carry Sxx to E_23 and E_13.
template <int P>
struct TriRot {
    static constexpr int NQ = (P + 1) * (P + 2) / 2;
    int s23[NQ], s13[NQ];
    constexpr TriRot() : s23(), s13() {
        for (int j = 0; j <= P; ++j)
            for (int i = 0; i + j <= P; ++i) {
                const int k = P - i - j, q = j * (P + 1) - j * (j - 1) / 2 + i;
                s23[q] = k * (P + 1) - k * (k - 1) / 2 + j;
                s13[q] = i * (P + 1) - i * (i - 1) / 2 + k;
            }
    }
};

// ---------------------------------------------------------------------------------------
// The paper's own element (Sec. 4.2): affine triangles with nq = (p+1)(p+2)/2 local nodes on
// the Blyth-Pozrikidis grid, single shot, owner-tile LDS accumulation with halo
// recomputation as in step_rows_kernel. nq consecutive lanes of a wave hold the nodes of one
// element (64 / nq elements per wave). Lane q gathers u at its node into the element's LDS
// stage and forms r_q = c^2 sum_m (g11 Sxx + g12 Sxy + g22 Syy)[q][m] (u_m - u_q), row q of the three
// reference matrices held in registers for the whole launch; the stage values are
// wave-uniform broadcasts. The element record is (g11, g12, g22, c^2), G = det J J^-1 J^-T
// constant over the element.
template <typename T, int P, int RB, int NP, bool GRAD>
__global__ void __attribute__((amdgpu_flat_work_group_size(RB, RB))) tri_rows_kernel(const StepArgs<T> a) {
    constexpr int NQ = (P + 1) * (P + 2) / 2;
    constexpr int NQP = (NQ + 3) & ~3;
    constexpr int EPW = 64 / NQ;
    constexpr int EPB = EPW * (RB / 64);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* stage = reinterpret_cast<T*>(smem_raw);          // [EPB][NQP]
    double* acc = reinterpret_cast<double*>(stage + EPB * NQP);
    T* pre_v = reinterpret_cast<T*>(acc + a.lds_own);
    T* pre_u = pre_v + a.lds_own;
    T* pre_m = pre_u + a.lds_own;

    const int tile = xcd_logical_block();
    const int nb = a.tile_nb[tile];
    const int nown = a.tile_nb[tile + 1] - nb;
    const int eb = a.tile_eb[tile];
    const int n_own_el = a.tile_eb[tile + 1] - eb;
    const int hb = a.halo_b[tile];
    const int n_items = n_own_el + (a.halo_b[tile + 1] - hb);
    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_u = make_rsrc(a.u_in, a.state_bytes);
    const rsrc_t r_pair = make_rsrc(a.u_pair, a.u_pair ? a.state_bytes : 0u);
    if (a.mode == 0) {
        const int ndw = nown * (int)(sizeof(T) / 4);
        const uint32_t off = (uint32_t)nb * (uint32_t)sizeof(T);
        lds_prefetch<RB>(make_rsrc(a.v, a.state_bytes), off, pre_v, ndw);
        lds_prefetch<RB>(r_u, off, pre_u, ndw);
        lds_prefetch<RB>(make_rsrc(a.dtminv, a.state_bytes), off, pre_m, ndw);
    }
    for (int i = threadIdx.x; i < nown; i += RB) acc[i] = 0.0;
    lds_barrier();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kw = lane / NQ, q = lane - kw * NQ;
    const int slot = wave * EPW + kw;
    T* st = stage + slot * NQP;
    // local node (i, j) of lane q (j outer, i inner); element-interior nodes have i, j, k >= 1
    int qi = q, qj = 0;
    while (qj <= P && qi >= P + 1 - qj) { qi -= P + 1 - qj; ++qj; }
    const bool interior = qi >= 1 && qj >= 1 && P - qi - qj >= 1;
    // Row q of Sxx = E_12 stays in registers for the launch. E_23 and E_13 are Sxx with rows
    // and columns permuted by s = s_23, s_13 (the vertex symmetry of the node set), so
    // (E u)_q = sum_m Sxx[s(q)][m] u_{s^-1(m)}: lane s(q) forms that sum from its own row and
    // the element's values read through s^-1, and lane q takes it with a lane shuffle. A lane
    // holds 21 matrix entries at p = 5 instead of 63.
    T s1[NQ];
    const int qrow = kw < EPW ? q : 0;
#pragma unroll
    for (int m = 0; m < NQ; ++m) s1[m] = a.tri_S[qrow * NQ + m];
    constexpr TriRot<P> rot{};
    // lanes s23(q), s13(q) of this element: nodes (qj, qk, qi) and (qk, qi, qj)
    const int qk = P - qi - qj;
    const int src23 = lane - q + qk * (P + 1) - qk * (qk - 1) / 2 + qj;
    const int src13 = lane - q + qi * (P + 1) - qi * (qi - 1) / 2 + qk;
    // NP passes at a time: every pass's node ids and records are requested first, then every
    // pass's gathers, so NP passes cost about one memory round trip, and the ids and records
    // of the next NP passes are requested before this group's compute. The loads are
    // unconditional (an inactive lane reads at the buffer's byte count, which returns 0
    // without touching memory), so the wait counts stay exact through the loop.
    auto fetch = [&](int base, int (&es)[NP], int (&node)[NP], bool (&act)[NP], T (&rec)[NP][4]) {
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int k = base + pp * EPB + slot;
            act[pp] = kw < EPW && k < n_items;
            // halo elements have copies of their rows after the E element rows, in the
            // order of the halo list, so no load stands before the id load
            es[pp] = k < n_own_el ? eb + k : (int)a.E + hb + (k - n_own_el);
            node[pp] = bload<int>(r_conn, act[pp] ? (uint32_t)(es[pp] * NQ + q) * 4u : a.conn_bytes);
            const uint32_t og = act[pp] ? (uint32_t)es[pp] * (uint32_t)(4 * sizeof(T)) : a.G_bytes;
            if constexpr (sizeof(T) == 4) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(r_G, og, 0, 0);
#pragma unroll
                for (int c = 0; c < 4; ++c) rec[pp][c] = __uint_as_float(v[c]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; c += 2) {
                    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r_G, og + 8u * c, 0, 0);
                    rec[pp][c] = __builtin_bit_cast(double, ((unsigned long long)v[1] << 32) | v[0]);
                    rec[pp][c + 1] = __builtin_bit_cast(double, ((unsigned long long)v[3] << 32) | v[2]);
                }
            }
        }
    };
    int es_n[NP], node_n[NP];
    bool act_n[NP];
    T rec_n[NP][4];
    fetch(0, es_n, node_n, act_n, rec_n);
    for (int base = 0; base < n_items; base += NP * EPB) {
        int es[NP], node[NP];
        bool act[NP];
        T rec[NP][4], uq[NP];
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            es[pp] = es_n[pp];
            node[pp] = node_n[pp];
            act[pp] = act_n[pp];
#pragma unroll
            for (int c = 0; c < 4; ++c) rec[pp][c] = rec_n[pp][c];
        }
#pragma unroll
        for (int pp = 0; pp < NP; ++pp)
            uq[pp] = bload<T>(r_u, act[pp] ? (uint32_t)node[pp] * (uint32_t)sizeof(T) : a.state_bytes);
        // keep the order gathers, next ids, compute: a gather moved after the next ids would
        // make the first stage write wait for those ids as well
        __builtin_amdgcn_sched_barrier(0);
        fetch(base + NP * EPB, es_n, node_n, act_n, rec_n);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int k = base + pp * EPB + slot;
            T dot = T(0);
            if (act[pp]) {
                const T u = uq[pp];
                wave_sync();                           // earlier reads of the stage are done
                st[q] = u;
                wave_sync();
                // Every row of the reference matrices sums to zero (K_e 1 = 0), so a row
                // applies to the differences from the lane's own value: the common part of the
                // element's values cancels before rounding and the rounded matrices keep the
                // exact null space (in FP32 the plain product drifts by the rounding of the row
                // sums, which acts on the mean field every step)
                T y12 = T(0), z23 = T(0), z13 = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    y12 += s1[m] * (st[m] - u);
                    z23 += s1[m] * (st[rot.s13[m]] - u);          // u read through s23^-1
                    z13 += s1[m] * (st[rot.s23[m]] - u);          // u read through s13^-1
                }
                const T y23 = __shfl(z23, src23, 64), y13 = __shfl(z13, src13, 64);
                const T r = rec[pp][0] * y12 + rec[pp][1] * y23 + rec[pp][2] * y13;    // (Khat_e u_e)_q
                if constexpr (GRAD) {
                    if (k < n_own_el) dot = r * bload<T>(r_pair, (uint32_t)node[pp] * (uint32_t)sizeof(T));
                }
                const int loc = node[pp] - nb;
                if ((unsigned)loc < (unsigned)nown) {
                    if (interior) acc[loc] = (double)(rec[pp][3] * r);
                    else atomicAdd(&acc[loc], (double)(rec[pp][3] * r));
                }
            }
            if constexpr (GRAD) {
                // every lane takes part: sum the element's nq lanes, one atomic per own element
                T tot = T(0);
                const int lead = (kw < EPW ? kw : 0) * NQ;
#pragma unroll
                for (int m = 0; m < NQ; ++m) tot += __shfl(dot, lead + m, 64);
                if (q == 0 && act[pp] && k < n_own_el) atomicAdd(&a.grad[es[pp]], (double)tot);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);                     // this wave's LDS prefetches landed
    __syncthreads();

    if (a.src_b != nullptr) {
        const int sb = a.src_b[tile], se = a.src_b[tile + 1];
        if (se > sb) {
            const T amp = (T)ricker(a.src_t, a.f0, a.t0);
            for (int i = sb + threadIdx.x; i < se; i += RB)
                if (a.src_shot[i] == a.shot) atomicAdd(&acc[a.src_loc[i]], -(double)(a.src_w[i] * amp));
            __syncthreads();
        }
    }
    if (a.inj != nullptr) {
        const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
        if (re > rb) {
            for (int i = rb + threadIdx.x; i < re; i += RB) {
                const T val = a.inj[(int64_t)a.rec_idx[i] * a.inj_cols + a.inj_col];
                atomicAdd(&acc[a.rec_loc[i]], -(double)(val * a.inj_scale));
            }
            __syncthreads();
        }
    }
    if (a.mode == 0) {
        for (int i = threadIdx.x; i < nown; i += RB) {
            const T vn = pre_v[i] - pre_m[i] * (T)acc[i];
            const T un = pre_u[i] + a.dt * vn;
            a.v[nb + i] = vn;
            a.u_out[nb + i] = un;
            acc[i] = (double)un;
        }
        if (a.trace != nullptr) {
            const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
            if (re > rb) {
                __syncthreads();
                for (int i = rb + threadIdx.x; i < re; i += RB)
                    a.trace[(int64_t)a.rec_idx[i] * a.trace_cols + a.trace_col] = (T)acc[a.rec_loc[i]];
            }
        }
    } else {
        for (int i = threadIdx.x; i < nown; i += RB)
            a.r_out[nb + i] = a.mode == 2 ? a.dtminv[nb + i] * (T)acc[i] : (T)acc[i];
    }
}

template <typename T, int P, int RB>
hipError_t launch_tri(int64_t n_tiles, const StepArgs<T>& a, hipStream_t st) {
    // FP32: two passes per group (107 VGPRs, four waves per SIMD; on the 250k-triangle p = 5
    // mesh one pass ran 6% slower and three 1% slower); FP64: one pass (two would drop to two
    // waves per SIMD)
    constexpr int NP = sizeof(T) == 4 ? 2 : 1;
    auto fn = a.grad != nullptr ? tri_rows_kernel<T, P, RB, NP, true> : tri_rows_kernel<T, P, RB, NP, false>;
    const size_t lds = tri_lds_bytes(P, RB, a.lds_own, sizeof(T));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)n_tiles), dim3(RB), lds, st, a);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_tri_t(int threads, int64_t n_tiles, const StepArgs<T>& a, hipStream_t st) {
    if constexpr (P % 2 == 0) {
        return hipErrorInvalidValue;                  // triangles run odd p only
    } else {
        switch (threads) {
            case 256: return launch_tri<T, P, 256>(n_tiles, a, st);
            case 512: return launch_tri<T, P, 512>(n_tiles, a, st);
            case 1024: return launch_tri<T, P, 1024>(n_tiles, a, st);
            default: return hipErrorInvalidValue;
        }
    }
}

template <typename T, int P, int SL>
hipError_t launch_one(int64_t n_tiles, size_t lds, const StepArgs<T>& a, hipStream_t st) {
    auto fn = step_kernel<T, P, SL>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int64_t blocks = n_tiles * a.n_slices;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <typename T, int P, int RB, int NP>
hipError_t launch_rows(int64_t n_tiles, size_t lds, const StepArgs<T>& a, hipStream_t st) {
    auto fn = a.grad != nullptr ? step_rows_kernel<T, P, RB, NP, true> : step_rows_kernel<T, P, RB, NP, false>;
    lds = rows_lds_bytes(P, RB, a.lds_own, sizeof(T));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)n_tiles), dim3(RB), lds, st, a);
    return hipGetLastError();
}

template <typename T, int P, int BT>
hipError_t launch_shots(int64_t n_tiles, size_t lds, const StepArgs<T>& a, hipStream_t st) {
    // FP32 forward steps run the instantiation without the pairing (113 VGPRs, four waves
    // per SIMD); the one with it has 89 VGPRs and five waves but ran 2.5% slower
    void (*fn)(const StepArgs<T>);
    if constexpr (sizeof(T) == 8) {
        fn = a.tile_nbd != nullptr ? step_shots_kernel<T, P, BT, true, true> : step_shots_kernel<T, P, BT, false, true>;
    } else {
        fn = a.tile_nbd != nullptr
                 ? (a.grad != nullptr ? step_shots_kernel<T, P, BT, true, true> : step_shots_kernel<T, P, BT, true, false>)
                 : (a.grad != nullptr ? step_shots_kernel<T, P, BT, false, true> : step_shots_kernel<T, P, BT, false, false>);
    }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)(n_tiles * a.n_slices)), dim3(BT), lds, st, a);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_p(int sl, int geo, int64_t nt, size_t lds, const StepArgs<T>& a, hipStream_t st) {
    if (geo >= kGeoTri) {
        if (sl != 1) return hipErrorInvalidValue;
        return launch_tri_t<T, P>(geo - kGeoTri, nt, a, st);
    }
    if (geo >= kGeoShots) {
        if (sl != 64) return hipErrorInvalidValue;
        switch (geo - kGeoShots) {
            case 256: return launch_shots<T, P, 256>(nt, lds, a, st);
            case 512: return launch_shots<T, P, 512>(nt, lds, a, st);
            case 1024: return launch_shots<T, P, 1024>(nt, lds, a, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (geo) {
        if (sl != 1) return hipErrorInvalidValue;
        // geo = threads per workgroup * 8 + passes batched per round of loads
        switch (geo) {
            case 256 * 8 + 1: return launch_rows<T, P, 256, 1>(nt, lds, a, st);
            case 256 * 8 + 2: return launch_rows<T, P, 256, 2>(nt, lds, a, st);
            case 256 * 8 + 4: return launch_rows<T, P, 256, 4>(nt, lds, a, st);
            case 512 * 8 + 1: return launch_rows<T, P, 512, 1>(nt, lds, a, st);
            case 512 * 8 + 2: return launch_rows<T, P, 512, 2>(nt, lds, a, st);
            case 1024 * 8 + 1: return launch_rows<T, P, 1024, 1>(nt, lds, a, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (sl) {
        case 1: return launch_one<T, P, 1>(nt, lds, a, st);
        case 2: return launch_one<T, P, 2>(nt, lds, a, st);
        case 4: return launch_one<T, P, 4>(nt, lds, a, st);
        case 8: return launch_one<T, P, 8>(nt, lds, a, st);
        case 16: return launch_one<T, P, 16>(nt, lds, a, st);
        case 32: return launch_one<T, P, 32>(nt, lds, a, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------------------
// First-order u-v system with Heun's scheme, one launch per step. At GLL point (i, j) of an
// element the reference derivatives of u give grad u = J^-T (d/dxi, d/deta) u (V-dot,
// Eq. v_change), and V enters R through A_xi = w_i w_j (Vx y_eta - Vy x_eta),
// A_eta = w_i w_j (Vy x_xi - Vx y_xi) (det J cancels): R(a, b) -= D(i, a) A_xi(i, b) and
// D(j, b) A_eta(a, j). R is summed into the tile's owned nodes in FP64 LDS words; the owned
// nodes then take their new U.
// Two instantiations: the predictor (CORR = FUSE = false), run only when the context holds no
// prediction for the current state, and the fused corrector (CORR = FUSE = true), once per step.
//   predictor: R(V^n); U~ = U^n + h M-bar^-1 (R + y(t_n)). V~ is not stored.
//   corrector (CORR): V~ = V^n + h grad U^n is formed again in registers for every
//     element the tile touches (its flux needs it); own elements write
//     V^{n+1} = V^n + h/2 (grad U^n + grad U~); R(V~);
//     U^{n+1} = U^n / 2 + U~ / 2 + h/2 M-bar^-1 (R + y(t_{n+1})).
//   FUSE (with CORR): also the next step's predictor. V^{n+1} is formed for the halo
//     elements too (U^n, U~ and V^n are complete before the launch), R(V^{n+1}) goes into a
//     second accumulator, and the owned nodes also take the next
//     U~ = U^{n+1} + h M-bar^-1 (R(V^{n+1}) + y(t_{n+1})) into u_pred: one launch per step.
// Forming V~ again costs the corrector a second gather of U, and saves writing V~ and reading
// it back (4 of the 10 element-local V words per local node and step).
// Lane layout of step_rows_kernel: p+1 lanes per element, lane j holds row j, a per-element
// LDS stage exchanges values across rows within the wave. V is element-major [E][2][nq], so
// a row's p+1 values of a component are contiguous.
template <typename T, int P, bool CORR, bool FUSE>
__global__ void __launch_bounds__(kRowBlock / 2) heun_rows_kernel(const HeunArgs<T> a) {
    constexpr int RB = kRowBlock / 2;                  // 512 threads
    constexpr int N = P + 1, NQ = N * N;
    constexpr int NQP = (NQ + 3) & ~3;
    constexpr int EPW = 64 / N;
    constexpr int EPB = EPW * (RB / 64);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* stage = reinterpret_cast<T*>(smem_raw);          // [EPB][NQP]
    double* acc = reinterpret_cast<double*>(stage + EPB * NQP);   // [owned nodes]
    // FUSE: R(V^{n+1}) of the next step's predictor, [owned nodes]
    double* acc2 = acc + a.lds_own;
    // U^n, U~ (corrector) and 1/M-bar of the owned nodes, staged for the update: [3][lds_own]
    // (FP32 only: in FP64 the extra LDS would halve the blocks resident per CU)
    constexpr bool PRE = sizeof(T) == 4;
    T* pre_0 = reinterpret_cast<T*>(acc + (FUSE ? 2 : 1) * a.lds_own);
    T* pre_1 = pre_0 + a.lds_own;
    T* pre_m = pre_1 + a.lds_own;
    const int tile = xcd_logical_block();
    const int nb = a.tile_nb[tile];
    const int nown = a.tile_nb[tile + 1] - nb;
    const int eb = a.tile_eb[tile];
    const int n_own_el = a.tile_eb[tile + 1] - eb;
    const int hb = a.halo_b[tile];
    const int n_items = n_own_el + (a.halo_b[tile + 1] - hb);
    const rsrc_t r_conn = make_rsrc(a.conn, a.conn_bytes);
    const rsrc_t r_G = make_rsrc(a.G, a.G_bytes);
    const rsrc_t r_u0 = make_rsrc(a.u0, a.state_bytes);
    const rsrc_t r_u1 = make_rsrc(CORR ? a.u1 : a.u0, a.state_bytes);
    if constexpr (PRE) {
        const int ndw = nown * (int)(sizeof(T) / 4);
        const uint32_t off = (uint32_t)nb * (uint32_t)sizeof(T);
        lds_prefetch<RB>(r_u0, off, pre_0, ndw);
        if constexpr (CORR) lds_prefetch<RB>(r_u1, off, pre_1, ndw);
        lds_prefetch<RB>(make_rsrc(a.minv_w, a.state_bytes), off, pre_m, ndw);
    }
    for (int i = threadIdx.x; i < nown; i += RB) {
        acc[i] = 0.0;
        if constexpr (FUSE) acc2[i] = 0.0;
    }
    lds_barrier();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kw = lane / N, j = lane - kw * N;
    const int slot = wave * EPW + kw;
    T* st = stage + slot * NQP;
    // FP32: row j and column j of D in registers, selected from the uniform kernel arguments
    // (indexing the arguments by the lane's row reloads them from memory for every element:
    // 9% of the FP32 step; in FP64 the ten extra registers cost 2%, so it reloads them)
    constexpr bool HOIST = sizeof(T) == 4;
    T Dj[N], DjT[N], xij = a.xi[0], wj = a.w[0];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        Dj[m] = a.D[m];
        DjT[m] = a.D[m * N];
    }
#pragma unroll
    for (int jj = 1; jj < N; ++jj)
        if (j == jj) {
#pragma unroll
            for (int m = 0; m < N; ++m) {
                Dj[m] = a.D[jj * N + m];
                DjT[m] = a.D[m * N + jj];
            }
            xij = a.xi[jj];
            wj = a.w[jj];
        }
    const T h = a.h, hh = T(0.5) * a.h;
    for (int base = 0; base < n_items; base += EPB) {
        const int k = base + slot;
        if (kw >= EPW || k >= n_items) continue;
        const bool own = k < n_own_el;
        const int e = own ? eb + k : a.halo[hb + k - n_own_el];
        int idx[N];
        load_ids<N>(r_conn, (uint32_t)(e * NQ + N * j) * 4u, idx);
        T bl[8];
        load_rec8(r_G, (uint32_t)e * 8u * (uint32_t)sizeof(T), bl);
        T vx[N], vy[N];
        const int64_t vrow = (int64_t)e * 2 * NQ + N * j;   // component 0 of row j
#pragma unroll
        for (int i = 0; i < N; ++i) {
            vx[i] = a.v0[vrow + i];
            vy[i] = a.v0[vrow + NQ + i];
        }
        // x_xi, y_xi at eta = xi_j are constant along the row; x_eta, y_eta depend on xi_i
        const T xs = bl[0] + bl[2] * xij, ys = bl[3] + bl[5] * xij;
        // R of the flux of (fx, fy) for this lane's row, summed into the accumulator A
        auto flux = [&](const T (&fx)[N], const T (&fy)[N], double* A) {
            T r[N], aeta[N];
#pragma unroll
            for (int aa = 0; aa < N; ++aa) r[aa] = T(0);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T xt = bl[1] + bl[2] * a.xi[i], yt = bl[4] + bl[5] * a.xi[i];
                const T wij = a.w[i] * wj;
                const T axi = wij * (fx[i] * yt - fy[i] * xt);
                aeta[i] = wij * (fy[i] * xs - fx[i] * ys);
                // along the row: R(aa, j) -= D(i, aa) A_xi(i, j)
#pragma unroll
                for (int aa = 0; aa < N; ++aa) r[aa] -= a.D[i * N + aa] * axi;
            }
            // across rows: R(aa, j) -= sum_m D(m, j) A_eta(aa, m), A_eta exchanged via the stage
            wave_sync();                               // earlier reads of the stage are done
#pragma unroll
            for (int i = 0; i < N; ++i) st[i + N * j] = aeta[i];
            wave_sync();
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const T dmj = HOIST ? DjT[m] : a.D[m * N + j];
#pragma unroll
                for (int aa = 0; aa < N; ++aa) r[aa] -= dmj * st[aa + N * m];
            }
            wave_sync();                               // before the stage is written again
            const bool inner_row = j > 0 && j < P;
#pragma unroll
            for (int aa = 0; aa < N; ++aa) {
                const int loc = idx[aa] - nb;
                if ((unsigned)loc < (unsigned)nown) {
                    if (aa > 0 && aa < P && inner_row) A[loc] = (double)r[aa];
                    else atomicAdd(&A[loc], (double)r[aa]);
                }
            }
        };
        if constexpr (CORR) {
            // grad u at (i, j) from this lane's row u[] and the other rows in the stage
            auto grad = [&](const T (&u)[N], int i, T& dx, T& dy) {
                const T xt = bl[1] + bl[2] * a.xi[i], yt = bl[4] + bl[5] * a.xi[i];
                T gxi = T(0), geta = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    gxi += a.D[i * N + m] * u[m];
                    geta += (HOIST ? Dj[m] : a.D[j * N + m]) * st[i + N * m];
                }
                const T inv = T(1) / (xs * yt - xt * ys);
                dx = (yt * gxi - ys * geta) * inv;
                dy = (xs * geta - xt * gxi) * inv;
            };
            T u[N], nx[N], ny[N];
#pragma unroll
            for (int i = 0; i < N; ++i) u[i] = bload<T>(r_u0, (uint32_t)idx[i] * (uint32_t)sizeof(T));
            wave_sync();
#pragma unroll
            for (int i = 0; i < N; ++i) st[i + N * j] = u[i];
            wave_sync();
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T dx, dy;
                grad(u, i, dx, dy);
                nx[i] = vx[i] + hh * dx;
                ny[i] = vy[i] + hh * dy;
                vx[i] += h * dx;                       // V~
                vy[i] += h * dy;
            }
            if (FUSE || own) {
#pragma unroll
                for (int i = 0; i < N; ++i) u[i] = bload<T>(r_u1, (uint32_t)idx[i] * (uint32_t)sizeof(T));
                wave_sync();
#pragma unroll
                for (int i = 0; i < N; ++i) st[i + N * j] = u[i];
                wave_sync();
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    T dx, dy;
                    grad(u, i, dx, dy);
                    nx[i] += hh * dx;                  // V^{n+1}
                    ny[i] += hh * dy;
                    if (own) {
                        a.v_out[vrow + i] = nx[i];
                        a.v_out[vrow + NQ + i] = ny[i];
                    }
                }
            }
            if constexpr (FUSE) flux(nx, ny, acc2);
        }
        flux(vx, vy, acc);
    }
    __builtin_amdgcn_s_waitcnt(0);                     // this wave's LDS prefetches landed
    __syncthreads();
    if (a.src_b != nullptr) {
        const int sb = a.src_b[tile], se = a.src_b[tile + 1];
        if (se > sb) {
            const T amp = (T)ricker(a.src_t, a.f0, a.t0);
            for (int i = sb + threadIdx.x; i < se; i += RB)
                if (a.src_shot[i] == 0) {
                    atomicAdd(&acc[a.src_loc[i]], (double)(a.src_w[i] * amp));
                    if constexpr (FUSE) atomicAdd(&acc2[a.src_loc[i]], (double)(a.src_w[i] * amp));
                }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nown; i += RB) {
        const int node = nb + i;
        T u0, u1, mi;
        if constexpr (PRE) {
            u0 = pre_0[i];
            u1 = CORR ? pre_1[i] : u0;
            mi = pre_m[i];
        } else {
            u0 = a.u0[node];
            u1 = CORR ? a.u1[node] : u0;
            mi = a.minv_w[node];
        }
        const T un = CORR ? T(0.5) * u0 + T(0.5) * u1 + hh * (mi * (T)acc[i]) : u0 + h * (mi * (T)acc[i]);
        a.u_out[node] = un;
        if constexpr (FUSE) a.u_pred[node] = un + h * (mi * (T)acc2[i]);   // next step's U~
        acc[i] = (double)un;
    }
    if (a.trace != nullptr) {
        const int rb = a.rec_b[tile], re = a.rec_b[tile + 1];
        if (re > rb) {
            __syncthreads();
            for (int i = rb + threadIdx.x; i < re; i += RB)
                a.trace[(int64_t)a.rec_idx[i] * a.trace_cols + a.trace_col] = (T)acc[a.rec_loc[i]];
        }
    }
}

template <typename T, int P>
hipError_t launch_heun_p(int mode, int64_t n_tiles, size_t lds, const HeunArgs<T>& a, hipStream_t st) {
    constexpr int RB = kRowBlock / 2;
    if (mode != 0 && mode != 2) return hipErrorInvalidValue;
    auto fn = mode == 2 ? heun_rows_kernel<T, P, true, true> : heun_rows_kernel<T, P, false, false>;
    lds = heun_lds_bytes(P, mode, a.lds_own, sizeof(T));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)n_tiles), dim3(RB), lds, st, a);
    return hipGetLastError();
}

// Border pass of the 64-shot atomic scatter: every border node's v is complete once the
// step launch has ended; u_out = u_in + dt v on its rows (one wave per node and 64-shot slice),
// then the traces of receivers at border nodes.
template <typename T>
__global__ void __launch_bounds__(kBlock) border_update_kernel(const StepArgs<T> a, const int32_t* nodes,
                                                               int64_t n_nodes) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t items = n_nodes * a.n_slices;
    for (int64_t k = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; k < items; k += nw) {
        const int64_t node = nodes[k / a.n_slices];
        const int64_t g = node * a.S + (k % a.n_slices) * 64 + lane;
        a.u_out[g] = a.u_in[g] + a.dt * a.v[g];
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) border_trace_kernel(const StepArgs<T> a, const int32_t* rec_idx,
                                                              const int32_t* rec_node, int32_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)n * a.S) return;
    const int64_t k = i / a.S, s = i % a.S;
    a.trace[(s * a.n_rec + rec_idx[k]) * a.trace_cols + a.trace_col] = a.u_out[(int64_t)rec_node[k] * a.S + s];
}

// ------------------------------------------------------------------ utility kernels
// internal state index i: node-major (node * S + s) or shot-major (s * N + node)
template <typename T>
__global__ void to_original_kernel(const T* in, T* out, const int32_t* n2o, int64_t N, int32_t S,
                                   bool shot_major) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * S) return;
    const int64_t node = shot_major ? i % N : i / S;
    const int64_t s = shot_major ? i / N : i - node * S;
    out[s * N + n2o[node]] = in[i];
}

template <typename T>
__global__ void from_original_kernel(const T* in, T* out, const int32_t* n2o, int64_t N, int32_t S,
                                     bool shot_major) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * S) return;
    const int64_t node = shot_major ? i % N : i / S;
    const int64_t s = shot_major ? i / N : i - node * S;
    out[i] = in[s * N + n2o[node]];
}

template <typename T>
__global__ void fill_kernel(T* x, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
__global__ void scale_kernel(T* x, double s, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = (T)((double)x[i] * s);
}

template <typename T>
__global__ void sumsq_kernel(const T* x, int64_t n, double* out) {
    __shared__ double part[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)x[i];
        s += v * v;
    }
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        atomicAdd(out, t);
    }
}

__global__ void grad_to_original_kernel(const double* acc, double* out, const int32_t* e2o, int64_t E,
                                        double scale) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < E) out[e2o[k]] = scale * acc[k];
}

inline unsigned grid_for(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned grid_stride(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

template <typename T>
hipError_t launch_step(int p, int sl, int geo, int64_t nt, size_t lds, const StepArgs<T>& a, hipStream_t st) {
    switch (p) {
        case 1: return launch_p<T, 1>(sl, geo, nt, lds, a, st);
        case 2: return launch_p<T, 2>(sl, geo, nt, lds, a, st);
        case 3: return launch_p<T, 3>(sl, geo, nt, lds, a, st);
        case 4: return launch_p<T, 4>(sl, geo, nt, lds, a, st);
        case 5: return launch_p<T, 5>(sl, geo, nt, lds, a, st);
        case 6: return launch_p<T, 6>(sl, geo, nt, lds, a, st);
        case 7: return launch_p<T, 7>(sl, geo, nt, lds, a, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_elems(int p, int threads, bool atomic, const StepArgs<T>& a, hipStream_t st) {
    switch (p) {
        case 1: return launch_elems_t<T, 1>(threads, atomic, a, st);
        case 2: return launch_elems_t<T, 2>(threads, atomic, a, st);
        case 3: return launch_elems_t<T, 3>(threads, atomic, a, st);
        case 4: return launch_elems_t<T, 4>(threads, atomic, a, st);
        case 5: return launch_elems_t<T, 5>(threads, atomic, a, st);
        case 6: return launch_elems_t<T, 6>(threads, atomic, a, st);
        case 7: return launch_elems_t<T, 7>(threads, atomic, a, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_node_update(const StepArgs<T>& a, int64_t n, hipStream_t st) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(node_update_kernel<T>, dim3((unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b))), dim3(kBlock), 0,
                       st, a, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_global_points(const StepArgs<T>& a, int phase, hipStream_t st) {
    const int n = phase == 0 ? (a.n_src_pts > a.n_rec_pts ? a.n_src_pts : a.n_rec_pts) : a.n_rec_pts;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(global_points_kernel<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a,
                       phase);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_border(const StepArgs<T>& a, const int32_t* nodes, int64_t n_nodes, const int32_t* rec_idx,
                         const int32_t* rec_node, int32_t n_rec, hipStream_t st) {
    if (n_nodes > 0) {
        const int64_t waves = n_nodes * a.n_slices;
        const int64_t b = (waves + kBlock / 64 - 1) / (kBlock / 64);
        hipLaunchKernelGGL(border_update_kernel<T>, dim3((unsigned)(b > 65536 ? 65536 : b)), dim3(kBlock), 0, st,
                           a, nodes, n_nodes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.trace != nullptr && n_rec > 0) {
        const int64_t t = (int64_t)n_rec * a.S;
        hipLaunchKernelGGL(border_trace_kernel<T>, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           a, rec_idx, rec_node, n_rec);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_nodes_to_original(const T* in, T* out, const int32_t* n2o, int64_t N, int32_t S,
                                    bool shot_major, hipStream_t st) {
    hipLaunchKernelGGL(to_original_kernel<T>, dim3(grid_for(N * S)), dim3(kBlock), 0, st, in, out, n2o, N, S,
                       shot_major);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nodes_from_original(const T* in, T* out, const int32_t* n2o, int64_t N, int32_t S,
                                      bool shot_major, hipStream_t st) {
    hipLaunchKernelGGL(from_original_kernel<T>, dim3(grid_for(N * S)), dim3(kBlock), 0, st, in, out, n2o, N, S,
                       shot_major);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_stride(n)), dim3(kBlock), 0, st, x, v, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(T* x, double s, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(scale_kernel<T>, dim3(grid_stride(n)), dim3(kBlock), 0, st, x, s, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sumsq(const T* x, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(sumsq_kernel<T>, dim3(grid_stride(n)), dim3(kBlock), 0, st, x, n, out);
    return hipGetLastError();
}

hipError_t launch_grad_to_original(const double* acc, double* out, const int32_t* e2o, int64_t E,
                                   double scale, hipStream_t st) {
    hipLaunchKernelGGL(grad_to_original_kernel, dim3(grid_for(E)), dim3(kBlock), 0, st, acc, out, e2o, E, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_heun_stage(int p, int mode, int64_t nt, size_t lds, const HeunArgs<T>& a,
                             hipStream_t st) {
    switch (p) {
        case 1: return launch_heun_p<T, 1>(mode, nt, lds, a, st);
        case 2: return launch_heun_p<T, 2>(mode, nt, lds, a, st);
        case 3: return launch_heun_p<T, 3>(mode, nt, lds, a, st);
        case 4: return launch_heun_p<T, 4>(mode, nt, lds, a, st);
        case 5: return launch_heun_p<T, 5>(mode, nt, lds, a, st);
        case 6: return launch_heun_p<T, 6>(mode, nt, lds, a, st);
        case 7: return launch_heun_p<T, 7>(mode, nt, lds, a, st);
        default: return hipErrorInvalidValue;
    }
}

#define SEM_INSTANTIATE(T)                                                                        \
    template hipError_t launch_step<T>(int, int, int, int64_t, size_t, const StepArgs<T>&, hipStream_t); \
    template hipError_t launch_nodes_to_original<T>(const T*, T*, const int32_t*, int64_t, int32_t,   \
                                                    bool, hipStream_t);                           \
    template hipError_t launch_nodes_from_original<T>(const T*, T*, const int32_t*, int64_t,        \
                                                      int32_t, bool, hipStream_t);                \
    template hipError_t launch_fill<T>(T*, T, int64_t, hipStream_t);                              \
    template hipError_t launch_scale<T>(T*, double, int64_t, hipStream_t);                        \
    template hipError_t launch_sumsq<T>(const T*, int64_t, double*, hipStream_t);                 \
    template hipError_t launch_heun_stage<T>(int, int, int64_t, size_t, const HeunArgs<T>&, hipStream_t); \
    template hipError_t launch_elems<T>(int, int, bool, const StepArgs<T>&, hipStream_t);         \
    template hipError_t launch_node_update<T>(const StepArgs<T>&, int64_t, hipStream_t);          \
    template hipError_t launch_global_points<T>(const StepArgs<T>&, int, hipStream_t);              \
    template hipError_t launch_border<T>(const StepArgs<T>&, const int32_t*, int64_t, const int32_t*,     \
                                         const int32_t*, int32_t, hipStream_t);

SEM_INSTANTIATE(float)
SEM_INSTANTIATE(double)

}  // namespace sem
