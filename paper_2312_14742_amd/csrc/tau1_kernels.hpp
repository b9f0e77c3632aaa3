// tau1_kernels.hpp -- per-node gather step kernel and the service kernels
// (geometry encode, state upload/readback, FP64 reductions, copy probe).
#pragma once

#include "tau1_args.hpp"

namespace tau1 {

// Sample owning a block of a per-node launch (samples sorted by block0).
__device__ __forceinline__ int sample_of_block(const SampleDev* s, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kGatherBlock = 256;

// ---------------------------------------------------------------------------
// Per-node gather step (pull form).  One thread per node; the node reads the
// pre-step (drho, v) of each source x - c_k (periodic wrap, then the solid
// test), forms the equilibrium of Eq. (3) minus its weight and accumulates
// density and momentum in direction order; a solid source is replaced by the
// node's own state with the opposite direction (halfway bounce-back, Eq. (11)).
// One reciprocal per node (division-saving algorithm).  Contraction into FMA
// is disabled so the FP64 instance reproduces plain IEEE evaluation.
// ---------------------------------------------------------------------------
template <int Q, int P>
__global__ __launch_bounds__(kGatherBlock) void k_gather(StepArgs a) {
#pragma clang fp contract(off)
    using St = Storage<P>;
    using S = typename St::S;
    using T = typename St::T;
    using L = Lattice<Q>;
    const int s = sample_of_block(a.samples, a.nsamples, blockIdx.x);
    const SampleDev& sd = a.samples[s];
    const int64_t i = (int64_t)(blockIdx.x - sd.block0) * kGatherBlock + threadIdx.x;
    if (i >= sd.n) return;
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const uint32_t* mask = reinterpret_cast<const uint32_t*>(a.base + sd.mask);
    if (solid_bit(mask, sd.words, ny, x, y, z)) return;

    const S* pre = reinterpret_cast<const S*>(a.base + sd.state[a.parity]);
    S* post = reinterpret_cast<S*>(a.base + sd.state[a.parity ^ 1]);
    const int64_t st = sd.stride;
    const T isr = inv_scale_rho<P>(a), isu = inv_scale_u<P>(a);
    const T d0 = St::load(pre, i, isr);
    const T v0x = St::load(pre + st, i, isu);
    const T v0y = St::load(pre + 2 * st, i, isu);
    const T v0z = St::load(pre + 3 * st, i, isu);

    T d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int cx = L::c[k].x, cy = L::c[k].y, cz = L::c[k].z;
        int sx = x - cx, sy = y - cy, sz = z - cz;
        sx += sx < 0 ? nx : 0; sx -= sx >= nx ? nx : 0;
        sy += sy < 0 ? ny : 0; sy -= sy >= ny ? ny : 0;
        sz += sz < 0 ? nz : 0; sz -= sz >= nz ? nz : 0;
        T ds, vx, vy, vz, ex, ey, ez;
        if (!solid_bit(mask, sd.words, ny, sx, sy, sz)) {
            const int64_t j = sx + (int64_t)nx * (sy + (int64_t)ny * sz);
            ds = St::load(pre, j, isr);
            vx = St::load(pre + st, j, isu);
            vy = St::load(pre + 2 * st, j, isu);
            vz = St::load(pre + 3 * st, j, isu);
            ex = (T)cx; ey = (T)cy; ez = (T)cz;
        } else {
            ds = d0; vx = v0x; vy = v0y; vz = v0z;
            ex = (T)-cx; ey = (T)-cy; ez = (T)-cz;
        }
        const T rho = (T)1 + ds;
        const T cu = (ex * vx + ey * vy) + ez * vz;
        const T vv = (vx * vx + vy * vy) + vz * vz;
        const T p = ((T)3 * cu + ((T)4.5 * cu) * cu) - (T)1.5 * vv;
        const T f = (T)weight<Q>(k) * (ds + rho * p);
        d += f;
        jx += (T)cx * f;
        jy += (T)cy * f;
        jz += (T)cz * f;
    }
    const T r = (T)1 / ((T)1 + d);
    const T ghx = gh_of<T>(a, 0), ghy = gh_of<T>(a, 1), ghz = gh_of<T>(a, 2);
    const T ux = jx * r + ghx, uy = jy * r + ghy, uz = jz * r + ghz;
    const T sr = scale_rho<P>(a), su = scale_u<P>(a);
    St::store(post, i, d, sr);
    St::store(post + st, i, ux + ghx, su);
    St::store(post + 2 * st, i, uy + ghy, su);
    St::store(post + 3 * st, i, uz + ghz, su);
}

// ---------------------------------------------------------------------------
// D2Q9 step of the validation workloads (nz = 1), one thread per node, pull
// form as k_gather, with node types: a wall source (type 1) returns the node's
// own equilibrium in the opposite direction (halfway bounce-back, Eq. (11));
// a moving wall (type 2) adds the wall's momentum to it,
//   f_k(x) = f_opp(k)(x) + 6 w_k rho(x) (c_k . u_wall).
// With a.xbc the fluid nodes of columns x = 0 and nx - 1 are constant-pressure
// nodes (Zou-He): the populations that would come from outside are unknown,
// the known ones fix rho u_x through
//   inlet:  rho_in u_x  = drho_in  - [f0 + f3 + f4 + 2 (f2 + f6 + f8)]
//   outlet: rho_out u_x = [f0 + f3 + f4 + 2 (f1 + f5 + f7)] - drho_out
// (values minus their weights), and the node's new state is (rho_b, u_x, 0).
// FP64 reproduces the oracle's roundings (contraction off).
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kGatherBlock) void k_d2q9(StepArgs a) {
#pragma clang fp contract(off)
    using St = Storage<P>;
    using S = typename St::S;
    using T = typename St::T;
    using L = Lattice<9>;
    const int s = sample_of_block(a.samples, a.nsamples, blockIdx.x);
    const SampleDev& sd = a.samples[s];
    const int64_t i = (int64_t)(blockIdx.x - sd.block0) * kGatherBlock + threadIdx.x;
    if (i >= sd.n) return;
    const int nx = sd.nx, ny = sd.ny;
    const int x = (int)(i % nx);
    const int y = (int)(i / nx);
    const uint8_t* type = a.base + sd.types;
    if (type[i]) return;

    const S* pre = reinterpret_cast<const S*>(a.base + sd.state[a.parity]);
    S* post = reinterpret_cast<S*>(a.base + sd.state[a.parity ^ 1]);
    const int64_t st = sd.stride;
    const T d0 = St::load(pre, i, (T)1);
    const T v0x = St::load(pre + st, i, (T)1);
    const T v0y = St::load(pre + 2 * st, i, (T)1);
    const T uwx = (T)a.uw[0], uwy = (T)a.uw[1];
    const bool pressure = a.xbc && (x == 0 || x == nx - 1);

    T f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = L::c[k].x, cy = L::c[k].y;
        int sx = x - cx, sy = y - cy;
        sy += sy < 0 ? ny : 0; sy -= sy >= ny ? ny : 0;
        if (a.xbc && (sx < 0 || sx >= nx)) {
            f[k] = 0;  // unknown of a pressure column; not used
            continue;
        }
        sx += sx < 0 ? nx : 0; sx -= sx >= nx ? nx : 0;
        const int64_t j = sx + (int64_t)nx * sy;
        const int tj = type[j];
        T ds, vx, vy, ex, ey;
        if (tj == 0) {
            ds = St::load(pre, j, (T)1);
            vx = St::load(pre + st, j, (T)1);
            vy = St::load(pre + 2 * st, j, (T)1);
            ex = (T)cx; ey = (T)cy;
        } else {
            ds = d0; vx = v0x; vy = v0y;
            ex = (T)-cx; ey = (T)-cy;
        }
        const T rho = (T)1 + ds;
        const T cu = ex * vx + ey * vy;
        const T vv = vx * vx + vy * vy;
        const T p = ((T)3 * cu + ((T)4.5 * cu) * cu) - (T)1.5 * vv;
        T fk = (T)weight<9>(k) * (ds + rho * p);
        if (tj == 2) {
            const T cw = (T)cx * uwx + (T)cy * uwy;
            fk += (T)6 * (T)weight<9>(k) * ((T)1 + d0) * cw;
        }
        f[k] = fk;
    }
    const T ghx = gh_of<T>(a, 0), ghy = gh_of<T>(a, 1);
    T d, ux, uy;
    if (pressure) {
        const bool inlet = x == 0;
        const T db = (T)(inlet ? a.din : a.dout);
        if (inlet) {
            const T sk = (f[0] + f[3] + f[4]) + (T)2 * ((f[2] + f[6]) + f[8]);
            ux = (db - sk) / ((T)1 + db) + ghx;
        } else {
            const T sk = (f[0] + f[3] + f[4]) + (T)2 * ((f[1] + f[5]) + f[7]);
            ux = (sk - db) / ((T)1 + db) + ghx;
        }
        d = db;
        uy = ghy;
    } else {
        T jx = 0, jy = 0;
        d = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            d += f[k];
            jx += (T)L::c[k].x * f[k];
            jy += (T)L::c[k].y * f[k];
        }
        const T r = (T)1 / ((T)1 + d);
        ux = jx * r + ghx;
        uy = jy * r + ghy;
    }
    St::store(post, i, d, (T)1);
    St::store(post + st, i, ux + ghx, (T)1);
    St::store(post + 2 * st, i, uy + ghy, (T)1);
    St::store(post + 3 * st, i, (T)0, (T)1);
}

// State upload: staging FP64 (drho0, u0) for nodes [i0, i0 + len) of one
// sample into both buffers; v = u + g/2; solid nodes get exact zeros.
template <int P>
__global__ void k_upload(StepArgs a, int s, const uint8_t* __restrict__ solid,
                         const double* __restrict__ drho0, const double* __restrict__ u0,
                         int64_t i0, int64_t len) {
    using St = Storage<P>;
    using S = typename St::S;
    using T = typename St::T;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    const SampleDev& sd = a.samples[s];
    const int64_t i = i0 + t;
    T d = 0, vx = 0, vy = 0, vz = 0;
    if (!solid[t]) {
        // widen/narrow from FP64 in the compute type, then add g/2 there
        d = drho0 ? (T)drho0[t] : (T)0;
        vx = (u0 ? (T)u0[t] : (T)0) + gh_of<T>(a, 0);
        vy = (u0 ? (T)u0[len + t] : (T)0) + gh_of<T>(a, 1);
        vz = (u0 ? (T)u0[2 * len + t] : (T)0) + gh_of<T>(a, 2);
    }
    const T sr = scale_rho<P>(a), su = scale_u<P>(a);
    const int x = (int)(i % sd.nx);
    const int y = (int)((i / sd.nx) % sd.ny);
    const int z = (int)(i / ((int64_t)sd.nx * sd.ny));
    const int64_t e = state_slot(a.base, sd, x, y, z, i);
    if (e < 0) return;  // all-solid chunk of the packed layout: no storage
    for (int b = 0; b < 2; ++b) {
        S* p = reinterpret_cast<S*>(a.base + sd.state[b]);
        St::store(p, e, d, sr);
        St::store(p + sd.stride, e, vx, su);
        St::store(p + 2 * sd.stride, e, vy, su);
        St::store(p + 3 * sd.stride, e, vz, su);
    }
}

// State readback: nodes [i0, i0 + len) of one sample, current buffer, into
// FP64 staging (drho | ux | uy | uz, each len values); u = v - g/2 in FP64;
// solid nodes read 0.  With phys_rho the first array holds rho = 1 + drho
// (formed in FP64; 1 at solid nodes) instead.  Counts non-finite fluid values
// into *bad.
template <int P>
__global__ void k_export(StepArgs a, int s, double* __restrict__ out, int64_t i0,
                         int64_t len, int* bad, int phys_rho) {
    using St = Storage<P>;
    using S = typename St::S;
    using T = typename St::T;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    const SampleDev& sd = a.samples[s];
    const int64_t i = i0 + t;
    const int x = (int)(i % sd.nx);
    const int y = (int)((i / sd.nx) % sd.ny);
    const int z = (int)(i / ((int64_t)sd.nx * sd.ny));
    const uint32_t* mask = reinterpret_cast<const uint32_t*>(a.base + sd.mask);
    double d = 0, ux = 0, uy = 0, uz = 0;
    if (!solid_bit(mask, sd.words, sd.ny, x, y, z)) {
        const S* p = reinterpret_cast<const S*>(a.base + sd.state[a.parity]);
        const int64_t e = state_slot(a.base, sd, x, y, z, i);  // a fluid node has a slot
        d = (double)St::load(p, e, inv_scale_rho<P>(a));
        ux = (double)St::load(p + sd.stride, e, inv_scale_u<P>(a)) - a.gh[0];
        uy = (double)St::load(p + 2 * sd.stride, e, inv_scale_u<P>(a)) - a.gh[1];
        uz = (double)St::load(p + 3 * sd.stride, e, inv_scale_u<P>(a)) - a.gh[2];
        if (!isfinite(d) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz))
            atomicAdd(bad, 1);
    }
    out[t] = phys_rho ? 1.0 + d : d;
    out[len + t] = ux;
    out[2 * len + t] = uy;
    out[3 * len + t] = uz;
}

// ---------------------------------------------------------------------------
// FP64 reductions (mass and permeability), deterministic: block b owns the
// contiguous node range [b*chunk, (b+1)*chunk); each thread sums its strided
// sub-sequence in order, each wave combines its lanes with a fixed butterfly
// of lane shuffles, and the block's first wave adds the four wave totals in
// wave order.  Partials: (sum drho, sum u_axis, fluid count, non-finite
// count) per block.  The same order on every run gives the same bits.
// ---------------------------------------------------------------------------
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kReduceWaves = kReduceThreads / 64;

// Sum over the 64 lanes of a wave by an xor butterfly: lane i adds lane
// i ^ m for m = 32, 16, ..., 1.  Both partners form the same sum (addition
// commutes exactly), so every lane ends with the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// The four sums of a block in wave order; valid in thread 0.
__device__ __forceinline__ void block_sum4(double (&acc)[4]) {
    __shared__ double sh[kReduceWaves][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[wave][c] = acc[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double t = sh[0][c];
            for (int w = 1; w < kReduceWaves; ++w) t += sh[w][c];
            acc[c] = t;
        }
}

template <int P>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partial(StepArgs a, int s, int axis,
                                                                   double* __restrict__ partial) {
    using St = Storage<P>;
    using S = typename St::S;
    const SampleDev& sd = a.samples[s];
    const int64_t chunk = (sd.n + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(beg + chunk, sd.n);
    const uint32_t* mask = reinterpret_cast<const uint32_t*>(a.base + sd.mask);
    const S* p = reinterpret_cast<const S*>(a.base + sd.state[a.parity]);
    const S* pu = p + (int64_t)(1 + axis) * sd.stride;
    double acc[4] = {0, 0, 0, 0};  // sum drho, sum u, fluid nodes, non-finite nodes
    for (int64_t i = beg + threadIdx.x; i < end; i += kReduceThreads) {
        const int x = (int)(i % sd.nx);
        const int y = (int)((i / sd.nx) % sd.ny);
        const int z = (int)(i / ((int64_t)sd.nx * sd.ny));
        if (solid_bit(mask, sd.words, sd.ny, x, y, z)) continue;
        const int64_t e = state_slot(a.base, sd, x, y, z, i);
        const double d = (double)St::load(p, e, inv_scale_rho<P>(a));
        const double u = (double)St::load(pu, e, inv_scale_u<P>(a)) - a.gh[axis];
        if (!isfinite(d) || !isfinite(u)) { acc[3] += 1; continue; }
        acc[0] += d;
        acc[1] += u;
        acc[2] += 1;
    }
    block_sum4(acc);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) partial[blockIdx.x * 4 + c] = acc[c];
}

}  // namespace tau1
