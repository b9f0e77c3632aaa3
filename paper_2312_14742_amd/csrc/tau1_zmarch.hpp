// tau1_zmarch.hpp -- z-march step kernel for gfx950 (the hot path).
//
// Work decomposition.  One wavefront owns G whole x-rows (G = 1, 2 or 4
// lane groups of Lg = 64/G lanes); lane gl of a group holds PX consecutive
// nodes x = gl*PX .. gl*PX + PX - 1 of its row, so nx = Lg * PX and the
// periodic wrap in x is a rotation inside the lane group.  The wave marches
// along z over a segment of planes [z0, z1), keeping the partial sums of three
// destination planes (z-1, z, z+1) in registers.
//
// Per source plane the wave reads the stored (drho, v) of its own row and of
// the rows y-1 and y+1 (those two are shared with the neighbouring waves and
// come mostly from L2) with coalesced vector loads, and for every source node
// forms the equilibrium of Eq. (3) (minus its weight) in each lattice
// direction and adds it -- weighted, with its momentum c_k -- into the partial
// sums of the destination x + c_k ("push" along x and z, "pull" from the two
// neighbour rows).  x-neighbours inside a lane are registers; across lanes
// they move with one DPP rotate (or a lane permute for 32-lane groups).  This
// is the node-local form of Eqs. (8)-(10): each node's new density and
// momentum are the sums of the equilibria its neighbours send it.
//
// Solid nodes hold exact zeros, so as sources they send nothing.  Halfway
// bounce-back (Eq. (11)) -- a population sent from fluid x towards a solid
// neighbour returns to x along the opposite direction -- touches only the
// ~10 % of fluid nodes next to a wall; the wave collects those nodes into a
// dense list in LDS, evaluates their returned populations one node per lane,
// and scatters the sums back (compaction instead of per-lane masking of all
// 18-26 directions).
//
// After plane z has received everything it is finalised with one reciprocal
// of the density (the division-saving form of the paper) and stored; solid
// nodes are never written.  Arithmetic is FP32; storage FP32, FP16 (power of
// two scaled) or BF16.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tau1_kernels.hpp"

namespace tau1 {

constexpr int kZrWaves = 4;                 // waves per workgroup
constexpr int kZrThreads = 64 * kZrWaves;
constexpr int kZrMaxPX = 9;

// Tile shapes the autotuner chooses among: z-segment length per work item.
constexpr int kNumTiles = 4;
constexpr int kTileLZ[kNumTiles] = {16, 32, 64, 128};

// (G, PX) variants compiled into the kernel; nx = (64 / G) * PX.
struct ZrVariant {
    int g, px;
};
constexpr int kNumVariants = 15;
constexpr ZrVariant kVariants[kNumVariants] = {
    {1, 1}, {1, 2}, {1, 3}, {1, 4}, {1, 5}, {1, 6}, {1, 7}, {1, 8},
    {2, 1}, {2, 3}, {2, 5}, {2, 7}, {2, 9}, {4, 1}, {4, 3}};

inline int zr_variant_for(int nx) {
    for (int v = 0; v < kNumVariants; ++v)
        if ((64 / kVariants[v].g) * kVariants[v].px == nx) return v;
    return -1;
}

// ---------------------------------------------------------------------------
// Lane moves inside a lane group of Lg = 64 / G lanes.
// up(v):   lane gl receives v from lane gl - 1 (wrapping), i.e. data moves +x
// down(v): lane gl receives v from lane gl + 1 (wrapping), data moves -x
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ float lane_up(float v) {
    const int iv = __builtin_bit_cast(int, v);
    int r;
    if constexpr (G == 1) {
        r = __builtin_amdgcn_update_dpp(0, iv, 0x13C, 0xf, 0xf, false);  // wave_ror:1
    } else if constexpr (G == 4) {
        r = __builtin_amdgcn_update_dpp(0, iv, 0x121, 0xf, 0xf, false);  // row_ror:1
    } else {
        const int lane = __lane_id();
        const int src = (lane & 32) | ((lane + 31) & 31);
        r = __builtin_amdgcn_ds_bpermute(src << 2, iv);
    }
    return __builtin_bit_cast(float, r);
}

template <int G>
__device__ __forceinline__ float lane_down(float v) {
    const int iv = __builtin_bit_cast(int, v);
    int r;
    if constexpr (G == 1) {
        r = __builtin_amdgcn_update_dpp(0, iv, 0x134, 0xf, 0xf, false);  // wave_rol:1
    } else if constexpr (G == 4) {
        r = __builtin_amdgcn_update_dpp(0, iv, 0x12F, 0xf, 0xf, false);  // row_ror:15
    } else {
        const int lane = __lane_id();
        const int src = (lane & 32) | ((lane + 1) & 31);
        r = __builtin_amdgcn_ds_bpermute(src << 2, iv);
    }
    return __builtin_bit_cast(float, r);
}

// Extended solid mask: each (y, z) row holds xwords 32-bit words whose bit b
// is the solid flag of node x = b - 1 taken periodically (so bit 0 is x = nx-1
// and bit nx+1 is x = 0).  A lane reads the PX + 2 bits around its nodes.
__device__ __forceinline__ uint32_t xmask_window(const uint32_t* __restrict__ xm, int64_t row,
                                                 int xwords, int b0) {
    const uint32_t* p = xm + row * xwords + (b0 >> 5);
    const uint64_t lo = p[0], hi = p[1];
    return (uint32_t)(((hi << 32) | lo) >> (b0 & 31));
}

template <int P, int PX>
struct RawRow {
    typename Storage<P>::T d[PX], vx[PX], vy[PX], vz[PX];
};

// Loads PX consecutive stored values of the four state arrays starting at
// node index i (a lane's slots) and widens them to FP32.
template <int P, int PX>
__device__ __forceinline__ void load_row(const typename Storage<P>::S* __restrict__ base,
                                         int64_t stride, int64_t i, float isr, float isu,
                                         RawRow<P, PX>& r) {
    using St = Storage<P>;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        r.d[j] = St::load(base, i + j, isr);
        r.vx[j] = St::load(base + stride, i + j, isu);
        r.vy[j] = St::load(base + 2 * stride, i + j, isu);
        r.vz[j] = St::load(base + 3 * stride, i + j, isu);
    }
}

// Per-source quantities: the equilibrium of Eq. (3) minus its weight in a
// direction with cu = c.v is w * (A + cu * (R3 + R45 * cu)) with
// A = drho - 1.5 rho v.v, R3 = 3 rho, R45 = 4.5 rho, rho = 1 + drho.
struct Src {
    float a, r3, r45, vx, vy, vz;
};

__device__ __forceinline__ Src make_src(float d, float vx, float vy, float vz) {
    Src s;
    const float rho = 1.0f + d;
    const float vv = vx * vx + vy * vy + vz * vz;
    s.a = __builtin_fmaf(-1.5f * rho, vv, d);
    s.r3 = 3.0f * rho;
    s.r45 = 4.5f * rho;
    s.vx = vx;
    s.vy = vy;
    s.vz = vz;
    return s;
}

template <int CX, int CY, int CZ>
__device__ __forceinline__ float feq_m(const Src& s) {
    float cu = 0.0f;
    if constexpr (CX != 0) cu = CX > 0 ? s.vx : -s.vx;
    if constexpr (CY != 0) cu = (CX != 0) ? (CY > 0 ? cu + s.vy : cu - s.vy) : (CY > 0 ? s.vy : -s.vy);
    if constexpr (CZ != 0)
        cu = (CX != 0 || CY != 0) ? (CZ > 0 ? cu + s.vz : cu - s.vz) : (CZ > 0 ? s.vz : -s.vz);
    return __builtin_fmaf(__builtin_fmaf(s.r45, cu, s.r3), cu, s.a);
}

// acc[plane][component][slot]; plane 0,1,2 = z-1, z, z+1 relative to the
// source plane; component 0..3 = drho, jx, jy, jz.
template <int PX>
struct Acc {
    float v[3][4][PX];
};

template <int CX, int CY, int CZ, int PX>
__device__ __forceinline__ void add_to(Acc<PX>& acc, int slot, float w, float u) {
    constexpr int p = CZ + 1;
    acc.v[p][0][slot] = __builtin_fmaf(w, u, acc.v[p][0][slot]);
    if constexpr (CX != 0) acc.v[p][1][slot] = __builtin_fmaf(CX * w, u, acc.v[p][1][slot]);
    if constexpr (CY != 0) acc.v[p][2][slot] = __builtin_fmaf(CY * w, u, acc.v[p][2][slot]);
    if constexpr (CZ != 0) acc.v[p][3][slot] = __builtin_fmaf(CZ * w, u, acc.v[p][3][slot]);
}

// Push the direction-k contribution of every slot of a source row whose
// directions have c_y == CY.
template <int Q, int K, int G, int PX>
__device__ __forceinline__ void push_dir(Acc<PX>& acc, const Src (&s)[PX], int zmask) {
    using L = Lattice<Q>;
    constexpr int CX = L::c[K].x, CY = L::c[K].y, CZ = L::c[K].z;
    // zmask selects which destination planes this step still needs
    if (!((zmask >> (CZ + 1)) & 1)) return;
    constexpr float w = (float)weight<Q>(K);
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const float u = feq_m<CX, CY, CZ>(s[j]);
        const int dst = j + CX;
        if (dst >= 0 && dst < PX) {
            add_to<CX, CY, CZ, PX>(acc, dst, w, u);
        } else if (dst == PX) {
            add_to<CX, CY, CZ, PX>(acc, 0, w, lane_up<G>(u));
        } else {
            add_to<CX, CY, CZ, PX>(acc, PX - 1, w, lane_down<G>(u));
        }
    }
}

template <int Q, int CYSEL, int G, int PX, int K = 1>
__device__ __forceinline__ void push_row(Acc<PX>& acc, const Src (&s)[PX], int zmask) {
    if constexpr (K < Q) {
        if constexpr (Lattice<Q>::c[K].y == CYSEL) push_dir<Q, K, G, PX>(acc, s, zmask);
        push_row<Q, CYSEL, G, PX, K + 1>(acc, s, zmask);
    }
}

// Bounce-back sums of one fluid node (one per worker lane): every direction k
// whose neighbour x + c_k is solid returns the node's own equilibrium in k
// along -c_k.  win[dy+1][dz+1] holds the solid bits around the node (bit 1 =
// the node itself).
template <int Q, int K = 1>
__device__ __forceinline__ void bounce_sum(const Src& s, const uint32_t (&win)[3][3], float& d,
                                           float& jx, float& jy, float& jz) {
    if constexpr (K < Q) {
        using L = Lattice<Q>;
        constexpr int CX = L::c[K].x, CY = L::c[K].y, CZ = L::c[K].z;
        constexpr float w = (float)weight<Q>(K);
        const bool solid = (win[CY + 1][CZ + 1] >> (1 + CX)) & 1u;
        const float u = solid ? w * feq_m<CX, CY, CZ>(s) : 0.0f;
        d += u;
        if constexpr (CX != 0) jx -= CX * u;
        if constexpr (CY != 0) jy -= CY * u;
        if constexpr (CZ != 0) jz -= CZ * u;
        bounce_sum<Q, K + 1>(s, win, d, jx, jy, jz);
    }
}

// Solid-neighbour bits (one per slot) of a lane from its nine row windows.
template <int Q, int PX, int K = 1>
__device__ __forceinline__ uint32_t neighbour_solid(const uint32_t (&win)[3][3]) {
    if constexpr (K < Q) {
        using L = Lattice<Q>;
        constexpr int CX = L::c[K].x, CY = L::c[K].y, CZ = L::c[K].z;
        return (win[CY + 1][CZ + 1] >> (1 + CX)) | neighbour_solid<Q, PX, K + 1>(win);
    } else {
        return 0u;
    }
}

__device__ __forceinline__ int wrapi(int a, int n) {
    a = a < 0 ? a + n : a;
    return a >= n ? a - n : a;
}

// position of the n-th (0-based) set bit of m (n < popcount(m))
__device__ __forceinline__ int nth_set_bit(uint64_t m, int n) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint64_t part = (m >> pos) & ((width == 64 ? ~0ull : ((1ull << width) - 1)));
        const int c = __builtin_popcountll(part);
        if (n >= c) {
            n -= c;
            pos += width;
        }
    }
    return pos;
}

// One work item: G rows starting at row-group rg, destination planes [z0, z1).
template <int Q, int P, int G, int PX>
__device__ __forceinline__ void zr_item(const StepArgs& a, const SampleDev& sd, int rg, int z0,
                                        int z1, float* __restrict__ lds) {
    using St = Storage<P>;
    using S = typename St::S;
    constexpr int Lg = 64 / G;
    constexpr uint32_t mPX = (1u << PX) - 1u;
    const int lane = __lane_id();
    const int grp = lane / Lg;
    const int gl = lane % Lg;
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const int y = rg * G + grp;
    const bool active = y < ny;
    const int yc = active ? y : ny - 1;
    const int ym = wrapi(yc - 1, ny), yp = wrapi(yc + 1, ny);
    const int x0 = gl * PX;
    const int64_t stride = sd.stride;
    const S* pre = reinterpret_cast<const S*>(a.base + sd.state[a.parity]);
    S* post = reinterpret_cast<S*>(a.base + sd.state[a.parity ^ 1]);
    const uint32_t* xm = reinterpret_cast<const uint32_t*>(a.base + sd.xmask);
    const int xw = sd.xwords;
    const float isr = inv_scale_rho<P>(a), isu = inv_scale_u<P>(a);
    const float sr = scale_rho<P>(a), su = scale_u<P>(a);
    const float gx = 2.0f * a.ghf[0], gy = 2.0f * a.ghf[1], gz = 2.0f * a.ghf[2];

    Acc<PX> acc;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < PX; ++j) acc.v[p][c][j] = 0.0f;

    uint32_t fluid_prev = 0;  // own-row fluid bits of plane zs - 1

    for (int zs = z0 - 1; zs <= z1; ++zs) {
        // destination planes zs-1, zs, zs+1 that belong to this segment
        const int zmask = ((zs - 1 >= z0 && zs - 1 < z1) ? 1 : 0) |
                          ((zs >= z0 && zs < z1) ? 2 : 0) |
                          ((zs + 1 >= z0 && zs + 1 < z1) ? 4 : 0);
        const int zc = wrapi(zs % nz, nz);
        const int zm = wrapi(zc - 1, nz), zp = wrapi(zc + 1, nz);
        const int yrow[3] = {ym, yc, yp};
        const int zrow[3] = {zm, zc, zp};
        uint32_t win[3][3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
                win[dy][dz] = xmask_window(xm, (int64_t)zrow[dz] * ny + yrow[dy], xw, x0);

        // ---- neighbour rows y-1 (their c_y = +1 directions) and y+1 (c_y = -1)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int yr = side == 0 ? ym : yp;
            const uint32_t fl = ~(win[side == 0 ? 0 : 2][1] >> 1) & mPX;
            RawRow<P, PX> raw;
            if (fl) {
                load_row<P, PX>(pre, stride, ((int64_t)zc * ny + yr) * nx + x0, isr, isu, raw);
            } else {
#pragma unroll
                for (int j = 0; j < PX; ++j) raw.d[j] = raw.vx[j] = raw.vy[j] = raw.vz[j] = 0.0f;
            }
            Src s[PX];
#pragma unroll
            for (int j = 0; j < PX; ++j) s[j] = make_src(raw.d[j], raw.vx[j], raw.vy[j], raw.vz[j]);
            if (side == 0)
                push_row<Q, 1, G, PX>(acc, s, zmask);
            else
                push_row<Q, -1, G, PX>(acc, s, zmask);
        }

        // ---- own row: c_y = 0 directions, rest, bounce-back
        const uint32_t fown = ~(win[1][1] >> 1) & mPX;
        RawRow<P, PX> raw;
        if (fown) {
            load_row<P, PX>(pre, stride, ((int64_t)zc * ny + yc) * nx + x0, isr, isu, raw);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j) raw.d[j] = raw.vx[j] = raw.vy[j] = raw.vz[j] = 0.0f;
        }
        {
            Src s[PX];
#pragma unroll
            for (int j = 0; j < PX; ++j) s[j] = make_src(raw.d[j], raw.vx[j], raw.vy[j], raw.vz[j]);
            push_row<Q, 0, G, PX>(acc, s, zmask);
            if (zmask & 2) {
                constexpr float w0 = (float)weight<Q>(0);
#pragma unroll
                for (int j = 0; j < PX; ++j) acc.v[1][0][j] = __builtin_fmaf(w0, s[j].a, acc.v[1][0][j]);
            }
        }

        if (zmask & 2) {
            // fluid nodes of this row with at least one solid neighbour
            const uint32_t bmask =
                active ? (fown & neighbour_solid<Q, PX>(win) & mPX) : 0u;
            uint64_t bal[PX];
            int total = 0;
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                bal[j] = __ballot((bmask >> j) & 1u);
                total += __builtin_popcountll(bal[j]);
            }
            if (total) {
                // dense copy of the wave's own-row state: lds[c][slot][lane]
                if (bmask) {
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        lds[(0 * PX + j) * 64 + lane] = raw.d[j];
                        lds[(1 * PX + j) * 64 + lane] = raw.vx[j];
                        lds[(2 * PX + j) * 64 + lane] = raw.vy[j];
                        lds[(3 * PX + j) * 64 + lane] = raw.vz[j];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int base = 0; base < total; base += 64) {
                    const int i = base + lane;
                    if (i < total) {
                        // entry i in slot-major order -> (slot, owner lane)
                        int slot = 0, rank = i, cum = 0;
                        uint64_t m = bal[0];
#pragma unroll
                        for (int j = 0; j < PX; ++j) {
                            const int c = __builtin_popcountll(bal[j]);
                            if (i >= cum && i < cum + c) {
                                slot = j;
                                rank = i - cum;
                                m = bal[j];
                            }
                            cum += c;
                        }
                        const int owner = nth_set_bit(m, rank);
                        const int oy = rg * G + owner / Lg;
                        const int ox = (owner % Lg) * PX + slot;
                        const int oym = wrapi(oy - 1, ny), oyp = wrapi(oy + 1, ny);
                        const int oyrow[3] = {oym, oy, oyp};
                        uint32_t w2[3][3];
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                            for (int dz = 0; dz < 3; ++dz)
                                w2[dy][dz] = xmask_window(xm, (int64_t)zrow[dz] * ny + oyrow[dy], xw, ox);
                        float* e = lds + slot * 64 + owner;
                        const Src s = make_src(e[0], e[PX * 64], e[2 * PX * 64], e[3 * PX * 64]);
                        float d = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
                        bounce_sum<Q>(s, w2, d, jx, jy, jz);
                        e[0] = d;
                        e[PX * 64] = jx;
                        e[2 * PX * 64] = jy;
                        e[3 * PX * 64] = jz;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (bmask) {
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        if ((bmask >> j) & 1u) {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                acc.v[1][c][j] += lds[(c * PX + j) * 64 + lane];
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }

        // ---- plane zs - 1 is complete: finalise and store (fluid slots only)
        if ((zmask & 1) && active && fluid_prev) {
            const int zo = wrapi(zc - 1, nz);
            const int64_t i0 = ((int64_t)zo * ny + yc) * nx + x0;
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                if ((fluid_prev >> j) & 1u) {
                    const float d = acc.v[0][0][j];
                    const float r = __builtin_amdgcn_rcpf(1.0f + d);
                    St::store(post, i0 + j, d, sr);
                    St::store(post + stride, i0 + j, __builtin_fmaf(acc.v[0][1][j], r, gx), su);
                    St::store(post + 2 * stride, i0 + j, __builtin_fmaf(acc.v[0][2][j], r, gy), su);
                    St::store(post + 3 * stride, i0 + j, __builtin_fmaf(acc.v[0][3][j], r, gz), su);
                }
            }
        }
        fluid_prev = fown;
        // rotate the destination planes
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                acc.v[0][c][j] = acc.v[1][c][j];
                acc.v[1][c][j] = acc.v[2][c][j];
                acc.v[2][c][j] = 0.0f;
            }
    }
}

// Work item (4 x int32): sample, row group, z-segment start, z-segment end.
// Workgroups are remapped so that each XCD walks a contiguous range of items
// (neighbouring rows share their y-1 / y+1 reads in that XCD's L2).
template <int Q, int P>
__global__ __launch_bounds__(kZrThreads) void k_zmarch(StepArgs a) {
    __shared__ float lds_all[kZrWaves][4 * kZrMaxPX * 64];
    const int wave = threadIdx.x >> 6;
    const int nwg = gridDim.x;
    const int b = blockIdx.x;
    // XCD-aware order: dispatch is round-robin over 8 XCDs
    const int per = (nwg + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int lb = xcd * per + k;
    const int nwaves = ((nwg + 7) / 8) * 8 * kZrWaves;
    for (int item = lb * kZrWaves + wave; item < a.ntiles; item += nwaves) {
        const int4 t = reinterpret_cast<const int4*>(a.tiles)[item];
        const SampleDev& sd = a.samples[t.x];
        float* lds = lds_all[wave];
        switch (sd.variant) {
#define TAU1_ZR_CASE(V, GG, PP)                                      \
    case V:                                                          \
        zr_item<Q, P, GG, PP>(a, sd, t.y, t.z, t.w, lds);            \
        break;
            TAU1_ZR_CASE(0, 1, 1)
            TAU1_ZR_CASE(1, 1, 2)
            TAU1_ZR_CASE(2, 1, 3)
            TAU1_ZR_CASE(3, 1, 4)
            TAU1_ZR_CASE(4, 1, 5)
            TAU1_ZR_CASE(5, 1, 6)
            TAU1_ZR_CASE(6, 1, 7)
            TAU1_ZR_CASE(7, 1, 8)
            TAU1_ZR_CASE(8, 2, 1)
            TAU1_ZR_CASE(9, 2, 3)
            TAU1_ZR_CASE(10, 2, 5)
            TAU1_ZR_CASE(11, 2, 7)
            TAU1_ZR_CASE(12, 2, 9)
            TAU1_ZR_CASE(13, 4, 1)
            TAU1_ZR_CASE(14, 4, 3)
#undef TAU1_ZR_CASE
            default:
                break;
        }
    }
}

// Extended-mask builder: row words of the periodic, one-bit-shifted mask.
__global__ void k_build_xmask(const uint32_t* __restrict__ mask, uint32_t* __restrict__ xm,
                              int nx, int words, int xwords, int64_t nrows) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * xwords) return;
    const int64_t r = t / xwords;
    const int w = (int)(t % xwords);
    const uint32_t* row = mask + r * words;
    uint32_t out = 0;
    for (int b = 0; b < 32; ++b) {
        const int e = w * 32 + b;  // extended bit e <-> x = e - 1 (periodic)
        if (e > nx + 1) break;
        int x = e - 1;
        x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
        out |= ((row[x >> 5] >> (x & 31)) & 1u) << b;
    }
    xm[t] = out;
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
inline int zr_xwords(int nx) { return (nx + 2 + 31) / 32 + 1; }

inline bool zmarch_precision_ok(int prec) { return prec == kF32 || prec == kF16 || prec == kBF16; }

inline bool zmarch_tile_ok(int, int prec, int tile) {
    return zmarch_precision_ok(prec) && tile >= 0 && tile < kNumTiles;
}

inline int zmarch_default_tile(int, int) { return 2; }  // z-segments of 64 planes

template <int Q, int P>
void* zmarch_fn() { return reinterpret_cast<void*>(&k_zmarch<Q, P>); }

inline void* pick_zmarch(int q, int p, int) {
    switch (q * 10 + p) {
        case 151: return zmarch_fn<15, kF32>();
        case 152: return zmarch_fn<15, kF16>();
        case 153: return zmarch_fn<15, kBF16>();
        case 191: return zmarch_fn<19, kF32>();
        case 192: return zmarch_fn<19, kF16>();
        case 193: return zmarch_fn<19, kBF16>();
        case 271: return zmarch_fn<27, kF32>();
        case 272: return zmarch_fn<27, kF16>();
        case 273: return zmarch_fn<27, kBF16>();
    }
    return nullptr;
}

inline int zmarch_threads(int) { return kZrThreads; }

// Resident-sized grid: at most enough workgroups for every item, rounded to
// whole XCD rounds.
inline int64_t zmarch_grid(int64_t nitems, int) {
    const int64_t wgs = (nitems + kZrWaves - 1) / kZrWaves;
    const int64_t cap = 256 * 8;  // 256 CUs x up to 8 workgroups resident
    int64_t g = wgs < cap ? wgs : cap;
    return (g + 7) / 8 * 8;
}

template <typename SH>
inline bool zmarch_supported(int, int prec, const SH* s, int n) {
    if (!zmarch_precision_ok(prec)) return false;
    for (int i = 0; i < n; ++i)
        if (s[i].dev.variant < 0) return false;
    return true;
}

inline void zmarch_tiling(SampleDev& sd) {
    sd.variant = zr_variant_for(sd.nx);
    sd.xwords = zr_xwords(sd.nx);
    const int g = sd.variant >= 0 ? kVariants[sd.variant].g : 1;
    sd.tiles_y = (sd.ny + g - 1) / g;
}

// Work list for z-segment length lz: items (sample, row group, z0, z1) with
// row groups fastest so neighbouring rows are neighbouring items.
template <typename SH>
inline std::vector<int32_t> zmarch_worklist(const SH* s, int n, int lz) {
    std::vector<int32_t> out;
    for (int i = 0; i < n; ++i) {
        const SampleDev& sd = s[i].dev;
        if (sd.variant < 0) continue;
        for (int z0 = 0; z0 < sd.nz; z0 += lz) {
            const int z1 = z0 + lz < sd.nz ? z0 + lz : sd.nz;
            for (int rg = 0; rg < sd.tiles_y; ++rg) {
                out.push_back(i);
                out.push_back(rg);
                out.push_back(z0);
                out.push_back(z1);
            }
        }
    }
    return out;
}

template <typename SH>
inline int64_t zmarch_max_items(const SH* s, int n) {
    int64_t items = 0;
    for (int i = 0; i < n; ++i) {
        const SampleDev& sd = s[i].dev;
        if (sd.variant < 0) continue;
        items += (int64_t)sd.tiles_y * ((sd.nz + kTileLZ[0] - 1) / kTileLZ[0]);
    }
    return items;
}

// Autotune cache: one line per entry "tau1 <arch> q<Q> p<P> n<bucket> tile <t> ms <x>".
inline int64_t size_bucket(int64_t n) {
    int64_t b = 1;
    while (b < n) b <<= 1;
    return b;
}

inline int zmarch_cache_lookup(const char* path, int q, int p, int64_t nodes) {
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int found = -1;
    const int64_t bucket = size_bucket(nodes);
    while (std::fgets(line, sizeof line, f)) {
        int qq, pp, tile;
        long long nb;
        float ms;
        char arch[64];
        if (std::sscanf(line, "tau1 %63s q%d p%d n%lld tile %d ms %f", arch, &qq, &pp, &nb, &tile,
                        &ms) == 6 &&
            std::strcmp(arch, "gfx950") == 0 && qq == q && pp == p && nb == bucket && tile >= 0 &&
            tile < kNumTiles)
            found = tile;
    }
    std::fclose(f);
    return found;
}

inline void zmarch_cache_store(const char* path, int q, int p, int64_t nodes, int tile, float ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "tau1 gfx950 q%d p%d n%lld tile %d ms %.6f\n", q, p,
                 (long long)size_bucket(nodes), tile, ms);
    std::fclose(f);
}

}  // namespace tau1
