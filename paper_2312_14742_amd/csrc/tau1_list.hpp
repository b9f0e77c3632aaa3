// tau1_list.hpp -- the per-node gather over a list of fluid nodes, for very
// porous-poor media: one thread per fluid node instead of one per node, so a
// wave holds fluid nodes only, however little of the lattice is fluid.
#pragma once

#include "tau1_kernels.hpp"

namespace tau1 {

// Fluid-node list of one sample, in the workspace: `list` is the byte offset
// of nf uint32 node indices (increasing); the launch gives the sample the
// blocks fblock0 .. fblock0 + ceil(nf / kGatherBlock) - 1.
struct ListDev {
    int64_t list;
    int64_t nf;
    int64_t fblock0;
};

__device__ __forceinline__ int sample_of_list_block(const ListDev* l, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (l[mid].fblock0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One step (pull form) at the listed fluid nodes.  The arithmetic and its
// order are those of k_gather (Eqs. (8)-(11), equilibria of Eq. (3) minus
// their weight, one reciprocal of rho), so both kernels give the same bits;
// only the node a thread takes differs.  Solid nodes are never visited: their
// stored zeros are written once at upload and never change.
template <int Q, int P>
__global__ __launch_bounds__(kGatherBlock) void k_gather_list(StepArgs a, const ListDev* ld) {
#pragma clang fp contract(off)
    using St = Storage<P>;
    using S = typename St::S;
    using T = typename St::T;
    using L = Lattice<Q>;
    const int s = sample_of_list_block(ld, a.nsamples, blockIdx.x);
    const ListDev& l = ld[s];
    const int64_t t = (int64_t)(blockIdx.x - l.fblock0) * kGatherBlock + threadIdx.x;
    if (t >= l.nf) return;
    const SampleDev& sd = a.samples[s];
    const int64_t i = reinterpret_cast<const uint32_t*>(a.base + l.list)[t];
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const uint32_t* mask = reinterpret_cast<const uint32_t*>(a.base + sd.mask);

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

}  // namespace tau1
