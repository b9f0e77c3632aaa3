// tau1_zmarch.hpp -- z-march step kernel for gfx950 (the hot path).
//
// Work decomposition.  One wavefront owns G whole x-rows (G = 1, 2 or 4
// lane groups of Lg = 64/G lanes).  A row is cut into C chunks of Lg*K nodes;
// lane gl of a group holds the K consecutive nodes gl*K .. gl*K + K - 1 of
// every chunk, so nx = C * Lg * K, each memory instruction of a group covers
// one contiguous chunk, and the periodic wrap in x is a rotation inside the
// lane group (plus a chunk hand-over at the group's first/last lane).  The
// wave marches along z over a segment of planes [z0, z1), keeping the partial
// sums of three destination planes (z-1, z, z+1) in registers.
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
// bounce-back (Eq. 11) -- a population sent from fluid x towards a solid
// neighbour returns to x along the opposite direction -- touches only the
// fluid nodes next to a wall (about 12 % of them at porosity 0.7).  A static
// per-row list of those nodes is built once at set-up; for each plane the
// wave evaluates the listed nodes one per lane and passes the sums through
// LDS to the lanes that own them (instead of masking all 18-26 directions of
// every node).
//
// After plane z has received everything it is finalised with one reciprocal
// of the density (the division-saving form of the paper) and stored; solid
// nodes are never written.  Arithmetic is FP32; storage FP32, FP16 (power of
// two scaled) or BF16.
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tau1_args.hpp"

// Multiply-adds fuse only where one expression writes a * b + c (and at the
// explicit fmaf calls), never across statements: every tile and load
// schedule then forms each sum with the same roundings, so results do not
// depend on the tile the autotuner picks.
#pragma clang fp contract(on)

namespace tau1 {

constexpr int kZrWaves = 4;                 // waves per workgroup
constexpr int kZrThreads = 64 * kZrWaves;

// Tile shapes the autotuner chooses among: z-segment length per work item
// (tile % 4) and the load schedule, tile / 4:
//   0  each source row is loaded just before it is used;
//   1  rows shared through LDS inside the workgroup (one-row-per-wave
//      layouts; rolling prefetch for the others);
//   2  rolling prefetch: row y-1 of the next plane is requested during this
//      plane;
//   3  as 1, for samples stored in the packed layout (only all-solid lane
//      chunks are left out of memory); the tiles of a context are those of
//      its layout: 0-2 dense, 3 packed.
// Tile 16 (packed layout only) is not a z-march: one lane per stored chunk
// (k_chunks), for media whose rows are mostly solid; it gives the same bits.
constexpr int kChunkTile = 16;
constexpr int kNumTiles = 17;
constexpr int kTileLZ[4] = {16, 32, 64, 128};
inline int tile_lz(int tile) { return kTileLZ[tile & 3]; }
inline int tile_mode(int tile) { return tile / 4; }
// Chunk tile: its work item (4 x int32) is sample, first packed chunk,
// number of chunks (at most 64, one wave), unused; its chunk list entry holds
// row y + ny z (bits 7..31) and chunk index in the row (bits 0..6).
constexpr int kCkWaves = 4;
constexpr int kCkThreads = 64 * kCkWaves;
constexpr int kChunkBits = 7;
inline bool tile_packed(int tile) { return tile_mode(tile) == 3 || tile == kChunkTile; }
// The z-march tile that stands in for the chunk tile in a launch group that
// is not packed (a batch may mix packed and dense lane layouts).
inline int tile_zmarch(int tile) { return tile == kChunkTile ? 14 : tile; }

// Load schedule of a (layout, mode) pair: shared rows need one row per wave.
constexpr bool zr_share(int g, int mode) { return (mode == 1 || mode == 3) && g == 1; }
constexpr bool zr_roll(int g, int mode) { return mode == 2 || ((mode == 1 || mode == 3) && g != 1); }
// Packed-layout rows (mode 3 exists only for one-row-per-wave layouts).
constexpr bool zr_packed(int g, int mode) { return mode == 3 && g == 1; }

// Lane layouts (G, C, K, L) compiled into the kernel: G rows per wave, each
// row in C chunks of L lanes x K nodes, nx = C * L * K.  L = 64 / G for the
// full layouts; the one-row layouts with L < 64 leave lanes L..63 idle (they
// load and store nothing) so that rows of 96, 160, 224 and 288 nodes get the
// one-row-per-wave schedules (rows shared through LDS, packed state) too.
struct ZrVariant {
    int g, c, k, l;
};
constexpr int kNumVariants = 15;
constexpr ZrVariant kVariants[kNumVariants] = {
    {1, 1, 1, 64}, {1, 1, 2, 64}, {1, 1, 3, 64}, {1, 1, 4, 64}, {1, 1, 5, 64}, {1, 2, 3, 64},
    {1, 2, 4, 64}, {2, 1, 1, 32}, {1, 1, 2, 48}, {1, 1, 4, 40}, {1, 1, 4, 56}, {1, 1, 6, 48},
    {4, 1, 1, 16}, {4, 1, 3, 16}, {4, 1, 5, 16}};

constexpr int zr_nx(const ZrVariant& v) { return v.c * v.l * v.k; }

inline int zr_variant_for(int nx) {
    for (int v = 0; v < kNumVariants; ++v)
        if (zr_nx(kVariants[v]) == nx) return v;
    return -1;
}

// ---------------------------------------------------------------------------
// Lane moves inside a lane group of L lanes (64 / G, or fewer for a one-row
// layout with idle lanes).  The DPP rotations give every lane a source, so
// they need no previous value of the destination (mov_dpp, not update_dpp).
// up(v):   lane gl receives v from lane gl - 1 (wrapping), i.e. data moves +x
// down(v): lane gl receives v from lane gl + 1 (wrapping), data moves -x
// Per-lane facts the moves need: the first and last lane of the group, and
// for L < 64 the byte addresses of the source lanes of a crossbar permute.
// ---------------------------------------------------------------------------
struct ZrLanes {
    // all ones on the group's first / last lane, else zero (bit masks for
    // the chunk hand-over: one bitwise select instead of a compare and a
    // conditional move)
    uint32_t first, last;
    int up, down;
};

// Per lane: a where the mask m is all ones, b where it is zero.
__device__ __forceinline__ float lane_pick(uint32_t m, float a, float b) {
    const uint32_t ia = __builtin_bit_cast(uint32_t, a), ib = __builtin_bit_cast(uint32_t, b);
    return __builtin_bit_cast(float, (ia & m) | (ib & ~m));
}

template <int G, int NL>
__device__ __forceinline__ float lane_up(float v, const ZrLanes& ln) {
    const int iv = __builtin_bit_cast(int, v);
    int r;
    if constexpr (G == 1 && NL < 64) {
        r = __builtin_amdgcn_ds_bpermute(ln.up, iv);
    } else if constexpr (G == 1) {
        r = __builtin_amdgcn_mov_dpp(iv, 0x13C, 0xf, 0xf, true);  // wave_ror:1
    } else if constexpr (G == 4) {
        r = __builtin_amdgcn_mov_dpp(iv, 0x121, 0xf, 0xf, true);  // row_ror:1
    } else {
        const int lane = __lane_id();
        const int src = (lane & 32) | ((lane + 31) & 31);
        r = __builtin_amdgcn_ds_bpermute(src << 2, iv);
    }
    return __builtin_bit_cast(float, r);
}

template <int G, int NL>
__device__ __forceinline__ float lane_down(float v, const ZrLanes& ln) {
    const int iv = __builtin_bit_cast(int, v);
    int r;
    if constexpr (G == 1 && NL < 64) {
        r = __builtin_amdgcn_ds_bpermute(ln.down, iv);
    } else if constexpr (G == 1) {
        r = __builtin_amdgcn_mov_dpp(iv, 0x134, 0xf, 0xf, true);  // wave_rol:1
    } else if constexpr (G == 4) {
        r = __builtin_amdgcn_mov_dpp(iv, 0x12F, 0xf, 0xf, true);  // row_ror:15
    } else {
        const int lane = __lane_id();
        const int src = (lane & 32) | ((lane + 1) & 31);
        r = __builtin_amdgcn_ds_bpermute(src << 2, iv);
    }
    return __builtin_bit_cast(float, r);
}

// Extended solid mask: each (y, z) row holds xwords 32-bit words whose bit b
// is the solid flag of node x = b - 1 taken periodically (so bit 0 is x = nx-1
// and bit nx+1 is x = 0).  A lane reads the K + 2 bits around each chunk.
__device__ __forceinline__ uint32_t xmask_window(const uint32_t* __restrict__ xm, int64_t row,
                                                 int xwords, int b0) {
    const uint32_t* p = xm + row * xwords + (b0 >> 5);
    const uint64_t lo = p[0], hi = p[1];
    return (uint32_t)(((hi << 32) | lo) >> (b0 & 31));
}

// ---------------------------------------------------------------------------
// Buffer access.  Each state array and the extended mask get a raw buffer
// resource; a row's start is the uniform (scalar) offset and a lane's chunk
// the per-lane offset, so no per-lane address arithmetic is needed.  A lane
// with nothing to read (an unused wall-list slot) uses an offset beyond the
// buffer's range: such loads return zeros without touching memory.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kOob = 0x7ff00000;  // voffset beyond every buffer (< 2 GiB checked on the host)

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// Loads B bytes (B a multiple of 2) at voff + soff into w (little endian).
template <int B>
__device__ __forceinline__ void buf_load_bytes(rsrc_t r, int voff, int soff, uint32_t (&w)[(B + 3) / 4]) {
    int o = 0;
#pragma unroll
    for (; o + 16 <= B; o += 16) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff + o, soff, 0);
        w[o / 4] = v[0]; w[o / 4 + 1] = v[1]; w[o / 4 + 2] = v[2]; w[o / 4 + 3] = v[3];
    }
    if constexpr (B % 16 >= 12) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, voff + o, soff, 0);
        w[o / 4] = v[0]; w[o / 4 + 1] = v[1]; w[o / 4 + 2] = v[2];
        o += 12;
    } else if constexpr (B % 16 >= 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff + o, soff, 0);
        w[o / 4] = v[0]; w[o / 4 + 1] = v[1];
        o += 8;
    } else if constexpr (B % 16 >= 4) {
        w[o / 4] = __builtin_amdgcn_raw_buffer_load_b32(r, voff + o, soff, 0);
        o += 4;
    }
    if constexpr (B % 4 == 2) w[o / 4] = __builtin_amdgcn_raw_buffer_load_b16(r, voff + o, soff, 0);
}

// Stores of the new state are non-temporal (streaming): they are not read
// again in this step, and the L2 keeps room for the source rows that three
// waves read in turn.
constexpr int kStoreNT = 2;

// Stores take the whole offset in the per-lane voffset and a constant-zero
// soffset.  With a register soffset the compiler assumes that a VALU write to
// the data VGPRs of a wide (more than 8-byte) buffer store right after the
// store is safe and inserts no wait state; on gfx950, with several waves per
// SIMD, the store then sometimes sends the new register value (the data
// VGPRs are read after the next VALU instruction has written them).  With a
// constant soffset the compiler keeps the required gap.

template <int B>
__device__ __forceinline__ void buf_store_bytes(rsrc_t r, int voff, int soff,
                                                const uint32_t (&w)[(B + 3) / 4]) {
    int o = 0;
#pragma unroll
    for (; o + 16 <= B; o += 16) {
        __attribute__((ext_vector_type(4))) unsigned v = {w[o / 4], w[o / 4 + 1], w[o / 4 + 2], w[o / 4 + 3]};
        __builtin_amdgcn_raw_buffer_store_b128(v, r, voff + soff + o, 0, kStoreNT);
    }
    if constexpr (B % 16 >= 12) {
        __attribute__((ext_vector_type(3))) unsigned v = {w[o / 4], w[o / 4 + 1], w[o / 4 + 2]};
        __builtin_amdgcn_raw_buffer_store_b96(v, r, voff + soff + o, 0, kStoreNT);
        o += 12;
    } else if constexpr (B % 16 >= 8) {
        __attribute__((ext_vector_type(2))) unsigned v = {w[o / 4], w[o / 4 + 1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff + soff + o, 0, kStoreNT);
        o += 8;
    } else if constexpr (B % 16 >= 4) {
        __builtin_amdgcn_raw_buffer_store_b32(w[o / 4], r, voff + soff + o, 0, kStoreNT);
        o += 4;
    }
    if constexpr (B % 4 == 2) __builtin_amdgcn_raw_buffer_store_b16((unsigned short)w[o / 4], r, voff + soff + o, 0, kStoreNT);
}

// K stored values of one array (one lane chunk) widened to FP32.
template <int P, int K>
__device__ __forceinline__ void load_chunk(rsrc_t r, int voff, int soff, float (&v)[K], float isc) {
    using St = Storage<P>;
    using S = typename St::S;
    constexpr int B = K * (int)sizeof(S);
    uint32_t w[(B + 3) / 4];
    buf_load_bytes<B>(r, voff, soff, w);
    S tmp[K];
    __builtin_memcpy(tmp, w, sizeof(tmp));
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = St::load(tmp, j, isc);
}

template <int P, int K>
__device__ __forceinline__ void store_chunk(rsrc_t r, int voff, int soff, const float (&v)[K], float sc) {
    using St = Storage<P>;
    using S = typename St::S;
    constexpr int B = K * (int)sizeof(S);
    S tmp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) St::store(tmp, j, v[j], sc);
    uint32_t w[(B + 3) / 4] = {};
    __builtin_memcpy(w, tmp, sizeof(tmp));
    buf_store_bytes<B>(r, voff, soff, w);
}

template <int PX>
struct RawRow {
    float d[PX], vx[PX], vy[PX], vz[PX];
};

// Per-source quantities: the equilibrium of Eq. (3) minus its weight in a
// direction with cu = c.v is w * (A + cu * (R3 + R45 * cu)) with
// A = drho - 1.5 rho v.v, R3 = 3 rho, R45 = 1.5 R3 (= 4.5 rho), rho = 1 + drho.
// R45 is always formed from R3, so a source shared as (A, R3, v) gives the
// same bits wherever it is evaluated.
struct Src {
    float a, r3, r45, vx, vy, vz;
};

__device__ __forceinline__ Src make_src(float d, float vx, float vy, float vz) {
    Src s;
    const float rho = 1.0f + d;
    const float vv = vx * vx + vy * vy + vz * vz;
    s.a = __builtin_fmaf(-1.5f * rho, vv, d);
    s.r3 = 3.0f * rho;
    s.r45 = 1.5f * s.r3;
    s.vx = vx;
    s.vy = vy;
    s.vz = vz;
    return s;
}

// Components of a source kept in a shared LDS row slot: A, R3, vx, vy, vz.
constexpr int kSlotComps = 5;

template <int CX, int CY, int CZ>
__device__ __forceinline__ float feq_m(const Src& s) {
    float cu = 0.0f;
    if constexpr (CX != 0) cu = CX > 0 ? s.vx : -s.vx;
    if constexpr (CY != 0) cu = (CX != 0) ? (CY > 0 ? cu + s.vy : cu - s.vy) : (CY > 0 ? s.vy : -s.vy);
    if constexpr (CZ != 0)
        cu = (CX != 0 || CY != 0) ? (CZ > 0 ? cu + s.vz : cu - s.vz) : (CZ > 0 ? s.vz : -s.vz);
    return __builtin_fmaf(__builtin_fmaf(s.r45, cu, s.r3), cu, s.a);
}

// Partial sums of one destination plane: [component][slot], components drho,
// jx, jy, jz.  Three planes (z-1, z, z+1 of the source plane) rotate roles.
template <int PX>
struct Plane {
    float v[4][PX];
};

template <int PX>
struct Planes {
    Plane<PX>& m;  // destination plane z - 1
    Plane<PX>& c;  // z
    Plane<PX>& p;  // z + 1
};

template <int CX, int CY, int CZ, int PX>
__device__ __forceinline__ void add_to(Planes<PX>& pl, int slot, float w, float u) {
    Plane<PX>& q = CZ < 0 ? pl.m : (CZ == 0 ? pl.c : pl.p);
    q.v[0][slot] = __builtin_fmaf(w, u, q.v[0][slot]);
    if constexpr (CX != 0) q.v[1][slot] = __builtin_fmaf(CX * w, u, q.v[1][slot]);
    if constexpr (CY != 0) q.v[2][slot] = __builtin_fmaf(CY * w, u, q.v[2][slot]);
    if constexpr (CZ != 0) q.v[3][slot] = __builtin_fmaf(CZ * w, u, q.v[3][slot]);
}

// Push the direction-KD contribution of every slot of a source row.  Slot
// (c, j) sends to (c, j + c_x); across a lane boundary the value rotates one
// lane inside the group, and the group's first/last lane takes it from the
// neighbouring chunk (the node after the last of chunk c is the first of c+1).
template <int Q, int KD, int G, int C, int K, int NL>
__device__ __forceinline__ void push_dir(Planes<C * K>& pl, const Src (&s)[C * K], int zmask,
                                         const ZrLanes& ln) {
    using L = Lattice<Q>;
    constexpr int CX = L::c[KD].x, CY = L::c[KD].y, CZ = L::c[KD].z;
    if (!((zmask >> (CZ + 1)) & 1)) return;
    constexpr float w = (float)weight<Q>(KD);
    float edge[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const float u = feq_m<CX, CY, CZ>(s[c * K + j]);
            const int dst = j + CX;
            if (dst >= 0 && dst < K) {
                add_to<CX, CY, CZ, C * K>(pl, c * K + dst, w, u);
            } else if (dst == K) {
                edge[c] = lane_up<G, NL>(u, ln);
            } else {
                edge[c] = lane_down<G, NL>(u, ln);
            }
        }
    }
    if constexpr (CX != 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float v = edge[c];
            if constexpr (C > 1) {
                if constexpr (CX > 0) v = lane_pick(ln.first, edge[(c + C - 1) % C], v);
                else v = lane_pick(ln.last, edge[(c + 1) % C], v);
            }
            add_to<CX, CY, CZ, C * K>(pl, CX > 0 ? c * K : c * K + K - 1, w, v);
        }
    }
}

template <int Q, int CYSEL, int G, int C, int K, int NL, int KD = 1>
__device__ __forceinline__ void push_row(Planes<C * K>& pl, const Src (&s)[C * K], int zmask,
                                         const ZrLanes& ln) {
    if constexpr (KD < Q) {
        if constexpr (Lattice<Q>::c[KD].y == CYSEL)
            push_dir<Q, KD, G, C, K, NL>(pl, s, zmask, ln);
        push_row<Q, CYSEL, G, C, K, NL, KD + 1>(pl, s, zmask, ln);
    }
}

// Bounce-back sums of one wall node (one per worker lane): every direction k
// whose neighbour x + c_k is solid returns the node's own equilibrium in k
// along -c_k.  Sums are kept per weight class and weighted at the end.
// link(k) is all ones when the neighbour x + c_k is solid, else zero (the
// step kernels keep the solid links in different forms).
template <int Q, int KD = 1, typename Link>
__device__ __forceinline__ void bounce_sum(const Src& s, const Link& link, float (&d)[3],
                                           float (&j)[3][3]) {
    if constexpr (KD < Q) {
        using L = Lattice<Q>;
        constexpr int CX = L::c[KD].x, CY = L::c[KD].y, CZ = L::c[KD].z;
        constexpr int cls = (CX != 0) + (CY != 0) + (CZ != 0) - 1;  // face, edge, corner
        const uint32_t m = link(KD);
        const float u = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, feq_m<CX, CY, CZ>(s)) & m);
        d[cls] += u;
        if constexpr (CX != 0) j[cls][0] -= CX * u;
        if constexpr (CY != 0) j[cls][1] -= CY * u;
        if constexpr (CZ != 0) j[cls][2] -= CZ * u;
        bounce_sum<Q, KD + 1>(s, link, d, j);
    }
}

// Weighted wall returns of one node: density and momentum (r[0], r[1..3]) of
// the populations its solid links send back.  The step kernels all add these
// four values to the node's sums at the same point, so they share this code.
template <int Q, typename Link>
__device__ __forceinline__ void wall_sums(const Src& sw, const Link& link, float (&r)[4]) {
    float sd[3] = {0.f, 0.f, 0.f};
    float sj[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    bounce_sum<Q>(sw, link, sd, sj);
    constexpr float wf = (float)Lattice<Q>::w_face, we = (float)Lattice<Q>::w_edge,
                    wc = (float)Lattice<Q>::w_corner;
    r[0] = wf * sd[0] + we * sd[1] + wc * sd[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) r[1 + a] = wf * sj[0][a] + we * sj[1][a] + wc * sj[2][a];
}

__device__ __forceinline__ int wrapi(int a, int n) {
    a = a < 0 ? a + n : a;
    return a >= n ? a - n : a;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Chunk-table entries and wall-list row offsets are read with scalar loads:
// both tables are constant while a step runs, and the row (hence the
// address) is wave-uniform.  A vector load whose value a scalar needs at once
// would make the wave wait for every memory operation it has in flight --
// the previous plane's stores included -- since loads and stores retire
// through one in-order counter.
typedef unsigned int ct_u4 __attribute__((ext_vector_type(4)));
// Chunk tile: neighbour-row record of a stored chunk (position ci of row r)
// for one of the nine rows r' = (y + dy, z + dz).  x: packed index of the
// first stored chunk at or after position ci of r' (bits 0..28), stored flags
// of positions ci - 1 (bit 29; 0 at ci = 0), ci (bit 30) and ci + 1 (bit 31;
// 0 at the row's last position).  y: at ci = 0 and at the last position, the
// packed index of the chunk across the periodic x boundary in r' (bits
// 0..28) and its stored flag (bit 31); else 0.
typedef unsigned int ck_rec_t __attribute__((ext_vector_type(2)));
constexpr unsigned kRecIndex = (1u << 29) - 1u;
typedef const __attribute__((address_space(4))) ct_u4 ctab_t;
typedef const __attribute__((address_space(4))) uint32_t wofs_t;

// Constants of one work item (one wave).
template <int P, int G, int C, int K>
struct ZrItem {
    static constexpr int Lg = 64 / G;
    static constexpr int PX = C * K;
    static constexpr int ES = (int)sizeof(typename Storage<P>::S);
    // state arrays drho | vx | vy | vz of the read and the written buffer; the
    // packed layout uses one resource per buffer over all four arrays
    // (pre[0], post[0]) and addresses array c at c * abytes
    rsrc_t pre[4], post[4], xm, wl;
    int abytes;
    int lane, gl;
    ZrLanes ln;     // lane-move facts (first / last lane, permute sources)
    bool active;
    int nx, ny, nz, xw, z0, z1;
    int y0, yc, ym, yp;
    int voff[C];   // byte offset of the lane's chunk c inside a row
    int woff[C];   // byte offset of the lane's mask window word, chunk c
    int wsh[C];    // bit of the chunk's first node minus one in that window
    float isr, isu, sr, su, gx, gy, gz;
    wofs_t* woffs;          // wall-list row offsets (scalar loads)
    float* lds_res;         // bounce-back sums [4][G * nx] of this wave
    // shared-row mode (one row per wave): the workgroup's row slots
    // [2 planes][kZrWaves waves][kSlotComps components][nx], this wave's index, and
    // whether rows y-1 / y+1 are the rows of the neighbouring waves
    float* lds_rows;
    int wave;
    bool share_m, share_p;
    ctab_t* ctab;  // packed layout: chunk table of the sample (C entries per row)
};

// Solid-bit window of the wave's own row in plane zc, one per chunk: bit b
// is the node chunk_start + b - 1.
template <int P, int G, int C, int K>
__device__ __forceinline__ void load_windows(const ZrItem<P, G, C, K>& it, int zc,
                                             uint32_t (&win)[C]) {
    const int roff = (zc * it.ny + it.yc) * it.xw * 4;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const auto v = G == 1 ? __builtin_amdgcn_raw_buffer_load_b64(it.xm, it.woff[c], roff, 0)
                              : __builtin_amdgcn_raw_buffer_load_b64(it.xm, it.woff[c] + roff, 0, 0);
        const uint64_t u = ((uint64_t)v[1] << 32) | v[0];
        win[c] = (uint32_t)(u >> it.wsh[c]);
    }
}

// Fluid flags of the lane's C * K nodes (bit c * K + j).
template <int C, int K>
__device__ __forceinline__ uint32_t fluid_bits(const uint32_t (&win)[C]) {
    constexpr uint32_t mK = (1u << K) - 1u;
    uint32_t f = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) f |= (~(win[c] >> 1) & mK) << (c * K);
    return f;
}

// One source row's state (C chunks of K nodes).  Whole chunks are read,
// solid nodes included (they hold zeros): every cache line is then read
// whole, which costs less than skipping all-solid chunks line by line.
template <int P, int G, int C, int K>
__device__ __forceinline__ void load_row(const ZrItem<P, G, C, K>& it, int row, RawRow<C * K>& r) {
    const int roff = row * it.nx * ZrItem<P, G, C, K>::ES;
    const int soff = G == 1 ? roff : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int vo = it.voff[c] + (G == 1 ? 0 : roff);
        float t0[K], t1[K], t2[K], t3[K];
        load_chunk<P, K>(it.pre[0], vo, soff, t0, it.isr);
        load_chunk<P, K>(it.pre[1], vo, soff, t1, it.isu);
        load_chunk<P, K>(it.pre[2], vo, soff, t2, it.isu);
        load_chunk<P, K>(it.pre[3], vo, soff, t3, it.isu);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            r.d[c * K + j] = t0[j];
            r.vx[c * K + j] = t1[j];
            r.vy[c * K + j] = t2[j];
            r.vz[c * K + j] = t3[j];
        }
    }
}

// A lane's chunks of one row's sources in an LDS slot [kSlotComps][nx] (one
// row per wave): the wave publishes its own row, and it and its neighbours
// read the sources back instead of forming them again.
template <int P, int G, int C, int K>
__device__ __forceinline__ void src_to_lds(const ZrItem<P, G, C, K>& it, float* slot,
                                           const RawRow<C * K>& r) {
    constexpr int RS = 64 * C * K;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float a[K], r3[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const Src t = make_src(r.d[c * K + j], r.vx[c * K + j], r.vy[c * K + j], r.vz[c * K + j]);
            a[j] = t.a;
            r3[j] = t.r3;
        }
        float* e = slot + c * 64 * K + it.gl * K;
        __builtin_memcpy(e, a, 4 * K);
        __builtin_memcpy(e + RS, r3, 4 * K);
        __builtin_memcpy(e + 2 * RS, &r.vx[c * K], 4 * K);
        __builtin_memcpy(e + 3 * RS, &r.vy[c * K], 4 * K);
        __builtin_memcpy(e + 4 * RS, &r.vz[c * K], 4 * K);
    }
}

template <int P, int G, int C, int K>
__device__ __forceinline__ void src_from_lds(const ZrItem<P, G, C, K>& it, const float* slot,
                                             Src (&s)[C * K]) {
    constexpr int RS = 64 * C * K;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float* e = slot + c * 64 * K + it.gl * K;
        float a[K], r3[K], vx[K], vy[K], vz[K];
        __builtin_memcpy(a, e, 4 * K);
        __builtin_memcpy(r3, e + RS, 4 * K);
        __builtin_memcpy(vx, e + 2 * RS, 4 * K);
        __builtin_memcpy(vy, e + 3 * RS, 4 * K);
        __builtin_memcpy(vz, e + 4 * RS, 4 * K);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            Src& t = s[c * K + j];
            t.a = a[j];
            t.r3 = r3[j];
            t.r45 = 1.5f * r3[j];
            t.vx = vx[j];
            t.vy = vy[j];
            t.vz = vz[j];
        }
    }
}

// Packed layout: the chunk-table entries of one row (wave-uniform).
template <int C>
struct RowTab {
    uint32_t lo[C], hi[C], rank[C];
};

template <int P, int G, int C, int K>
__device__ __forceinline__ void row_tab(const ZrItem<P, G, C, K>& it, int row, RowTab<C>& t) {
    ctab_t* e = it.ctab + (int64_t)row * C;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const ct_u4 v = e[c];
        t.lo[c] = v.x;
        t.hi[c] = v.y;
        t.rank[c] = v.z;
    }
}

// Byte offsets of the lane's chunks of a packed row: the chunk's rank among
// the row group's fluid chunks (lanes below it with a set bit) added to the
// group's first packed index; an all-solid chunk gets the out-of-range offset,
// so its loads read zeros and its stores are dropped.
template <int P, int G, int C, int K>
__device__ __forceinline__ void chunk_voffs(const ZrItem<P, G, C, K>& it, const RowTab<C>& t,
                                            int (&vo)[C]) {
    constexpr uint32_t CB = (uint32_t)(K * ZrItem<P, G, C, K>::ES);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(t.hi[c], __builtin_amdgcn_mbcnt_lo(t.lo[c], 0u));
        const uint64_t bits = ((uint64_t)t.hi[c] << 32) | t.lo[c];
        vo[c] = ((bits >> it.lane) & 1u) ? (int)((t.rank[c] + below) * CB) : kOob;
    }
}

// One packed source row (whole chunks at the offsets vo).
template <int P, int G, int C, int K>
__device__ __forceinline__ void load_row_pk(const ZrItem<P, G, C, K>& it, const int (&vo)[C],
                                            RawRow<C * K>& r) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float t0[K], t1[K], t2[K], t3[K];
        load_chunk<P, K>(it.pre[0], vo[c], 0, t0, it.isr);
        load_chunk<P, K>(it.pre[0], vo[c], it.abytes, t1, it.isu);
        load_chunk<P, K>(it.pre[0], vo[c], 2 * it.abytes, t2, it.isu);
        load_chunk<P, K>(it.pre[0], vo[c], 3 * it.abytes, t3, it.isu);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            r.d[c * K + j] = t0[j];
            r.vx[c * K + j] = t1[j];
            r.vy[c * K + j] = t2[j];
            r.vz[c * K + j] = t3[j];
        }
    }
}

// Packed-layout state carried along the march: the lane's chunk offsets in
// the edge rows y-1 / y+1 of the current plane (their table entries are
// fetched one plane ahead) and in the own row of planes zs-1 (stored in this
// step) and zs.
template <int C>
struct PkPipe {
    int vm[C], vp[C];
    int vst[C], vcur[C];
};

// Wall-list state carried along the march: row offsets of the planes ahead
// (scalars) and the first 64 entries of the next plane (one per lane), loaded
// one plane ahead so the bounce-back never waits on memory.
template <int Q>
struct WallPipe {
    using E = typename WallEntry<Q>::type;
    int cur0, cur1;    // entries [cur0, cur1) of the current plane
    int next0, next1;  // of the next plane
    E cur;             // entry cur0 + lane, or 0
};

template <int P, int G, int C, int K>
__device__ __forceinline__ void wall_offsets(const ZrItem<P, G, C, K>& it, int plane, int& o0,
                                             int& o1) {
    const int zc = wrapi(plane % it.nz, it.nz);
    const int ng = G < it.ny - it.y0 ? G : it.ny - it.y0;
    if (ng <= 0) {
        // a padding row group past the lattice (shared-row blocks): no wall
        // nodes, and no row offsets to read
        o0 = o1 = 0;
        return;
    }
    const int r0 = zc * it.ny + it.y0;
    o0 = (int)it.woffs[r0];
    o1 = (int)it.woffs[r0 + ng];
}

template <int Q>
__device__ __forceinline__ typename WallEntry<Q>::type wall_load(rsrc_t wl, int idx, bool ok) {
    using E = typename WallEntry<Q>::type;
    const int vo = ok ? idx * (int)sizeof(E) : kOob;
    if constexpr (sizeof(E) == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(wl, vo, 0, 0);
        return ((uint64_t)v[1] << 32) | v[0];
    } else {
        return __builtin_amdgcn_raw_buffer_load_b32(wl, vo, 0, 0);
    }
}

// One stored value (at voff + soff) widened to FP32.
template <int P>
__device__ __forceinline__ float load_one(rsrc_t r, int voff, int soff, float isc) {
    using St = Storage<P>;
    using S = typename St::S;
    S tmp[1];
    if constexpr (sizeof(S) == 4) {
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        __builtin_memcpy(tmp, &w, 4);
    } else {
        const unsigned short w = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
        __builtin_memcpy(tmp, &w, 2);
    }
    return St::load(tmp, 0, isc);
}

// Stored state of the node of wall-list entry e (widened to FP32), for the
// bounce-back worker lane; e's row is the wave's row y0 + (e >> 10 & 3) of
// plane zc.
template <int Q, int P, int G, int C, int K>
__device__ __forceinline__ void wall_state(const ZrItem<P, G, C, K>& it, typename WallEntry<Q>::type e,
                                           int zc, bool ok, float (&v)[4]) {
    constexpr int ES = ZrItem<P, G, C, K>::ES;
    const int x = (int)(e & 1023u);
    const int row = zc * it.ny + it.y0;
    const int n = (int)((e >> 10) & 3u) * it.nx + x;  // node from the first row's start
    const int vo = ok ? n * ES : kOob;
    const int so = row * it.nx * ES;
    v[0] = load_one<P>(it.pre[0], vo, so, it.isr);
    v[1] = load_one<P>(it.pre[1], vo, so, it.isu);
    v[2] = load_one<P>(it.pre[2], vo, so, it.isu);
    v[3] = load_one<P>(it.pre[3], vo, so, it.isu);
}

// Halfway bounce-back (Eq. 11) at the wall nodes of this wave's rows in the
// current plane.  Lane i evaluates list entry i: the node's own equilibrium
// in every direction k whose neighbour x + c_k is solid, returned to the node
// along -c_k.  The node's state comes from the owners' LDS copy; the sums go
// through LDS back to the owners, which add them to the plane's partial sums
// and clear their slots for the next plane.
//
// Shared-row mode (state != nullptr): the node's source terms come from the
// wave's own row slot in LDS, and the sums go through `res`, a slot the owners
// clear first.  Otherwise the state of the first 64 nodes is v0 (loaded at the
// start of the step), later ones are loaded here, and `res` is the wave's
// sum area, which the owners clear after reading.
template <int Q, int P, int G, int C, int K>
__device__ __forceinline__ void bounce_list(const ZrItem<P, G, C, K>& it, Plane<C * K>& pc,
                                            const WallPipe<Q>& wp, int zc, const float (&v0)[4],
                                            const float* state, float* res) {
    constexpr int PX = C * K;
    constexpr int Lg = 64 / G;
    constexpr int RS = 64 * PX;  // = G * nx
    const int total = wp.cur1 - wp.cur0;
    const int grp = G == 1 ? 0 : it.lane / Lg;
    if (state) {
#pragma unroll
        for (int comp = 0; comp < 4; ++comp)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float z[K] = {};
                __builtin_memcpy(res + comp * RS + grp * (C * Lg * K) + c * Lg * K + it.gl * K, z,
                                 sizeof z);
            }
        __builtin_amdgcn_wave_barrier();
    }
    for (int base = 0; base < total; base += 64) {
        const int i = base + it.lane;
        typename WallEntry<Q>::type e = wp.cur;
        float v[4] = {v0[0], v0[1], v0[2], v0[3]};
        if (base > 0) {
            e = wall_load<Q>(it.wl, wp.cur0 + i, i < total);
            if (!state) wall_state<Q>(it, e, zc, i < total, v);
        }
        if (i < total) {
            const int n = (int)((e >> 10) & 3u) * it.nx + (int)(e & 1023u);
            const uint32_t links = (uint32_t)(e >> 12);
            Src sw;
            if (state) {
                sw.a = state[n];
                sw.r3 = state[RS + n];
                sw.r45 = 1.5f * sw.r3;
                sw.vx = state[2 * RS + n];
                sw.vy = state[3 * RS + n];
                sw.vz = state[4 * RS + n];
            } else {
                sw = make_src(v[0], v[1], v[2], v[3]);
            }
            float r[4];
            // bit k - 1 of the entry's links: the neighbour x + c_k is solid
            wall_sums<Q>(sw, [&](int k) { return (uint32_t)__builtin_amdgcn_sbfe((int)links, k - 1, 1); }, r);
#pragma unroll
            for (int c = 0; c < 4; ++c) res[c * RS + n] = r[c];
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int comp = 0; comp < 4; ++comp)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float* e = res + comp * RS + grp * (C * Lg * K) + c * Lg * K + it.gl * K;
            float t[K];
            __builtin_memcpy(t, e, sizeof t);
#pragma unroll
            for (int j = 0; j < K; ++j) pc.v[comp][c * K + j] += t[j];
            if (!state) {
                const float z[K] = {};
                __builtin_memcpy(e, z, sizeof z);
            }
        }
    __builtin_amdgcn_wave_barrier();
}

// One source plane zs: pl.m, pl.c, pl.p are the destination planes zs-1, zs,
// zs+1 (pl.p starts empty).  Finalises and stores plane zs-1 at the end.
//
// Load schedules (MODE, the tile's mode).  Mode 0: each source row is
// loaded just before it is used.  Shared rows (mode 1, one row per wave):
// each wave loads only its own row (requested at the end of the previous
// plane, `ahead`), publishes it in an LDS slot, and after one workgroup
// barrier per plane reads rows y-1 / y+1 from its neighbours' slots; only the
// block's edge rows come from memory.  Mode 3 is mode 1 on the packed layout:
// rows are read and written at their chunks' packed offsets.  Rolling
// prefetch (mode 2, and modes 1 and 3 with G > 1): the own row of the next
// plane (`ahead`) is requested during this plane.
template <int Q, int P, int G, int C, int K, int NL, int MODE, bool EARLY_OK>
__device__ __forceinline__ void zr_step(const ZrItem<P, G, C, K>& it, int zs, Planes<C * K> pl,
                                        uint32_t (&win_next)[C], uint32_t& fluid_prev,
                                        WallPipe<Q>& wp, RawRow<C * K>& ahead, PkPipe<C>& pk) {
    constexpr int PX = C * K;
    constexpr bool SHARE = zr_share(G, MODE);
    constexpr bool ROLL = zr_roll(G, MODE);
    constexpr bool PK = zr_packed(G, MODE);
    constexpr int RS = 64 * PX;
    const int z0 = it.z0, z1 = it.z1, ny = it.ny, nz = it.nz;
    const int zmask = ((zs - 1 >= z0 && zs - 1 < z1) ? 1 : 0) |
                      ((zs >= z0 && zs < z1) ? 2 : 0) |
                      ((zs + 1 >= z0 && zs + 1 < z1) ? 4 : 0);
    const int zc = wrapi(zs % nz, nz);
    const uint32_t fown = fluid_bits<C, K>(win_next);
    const int rm_ = zc * ny + it.ym, rp_ = zc * ny + it.yp, ro_ = zc * ny + it.yc;
    RawRow<PX> rm, rp, ro;
    // next plane's windows (also after the segment's last plane: a periodic,
    // in-range read; unconditional so that no load count depends on a branch)
    load_windows(it, wrapi((zs + 1) % nz, nz), win_next);
    // wall list one plane ahead: entries of plane zs + 1, offsets of zs + 2
    const auto e_next = wall_load<Q>(it.wl, wp.next0 + it.lane, it.lane < wp.next1 - wp.next0);
    int nn0, nn1;
    wall_offsets(it, zs + 2, nn0, nn1);
    // packed layout: chunk tables of the next plane's own and edge rows
    RowTab<C> tn_own, tn_m, tn_p;
    if constexpr (PK) {
        const int zn = wrapi((zs + 1) % nz, nz) * ny;
        row_tab(it, zn + it.yc, tn_own);
        row_tab(it, zn + it.ym, tn_m);
        row_tab(it, zn + it.yp, tn_p);
    }
    // state of this plane's first 64 wall nodes, used by the bounce-back below
    float wv[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (!SHARE)
        wall_state<Q>(it, wp.cur, zc, (zmask & 2) && it.lane < wp.cur1 - wp.cur0, wv);

    float* own = nullptr;
    float* spare = nullptr;
    int vn[C];  // packed layout: the lane's chunk offsets in the next plane's own row
    if constexpr (SHARE) {
        // slots of this plane (parity of zs) and of the next one
        const int b = zs & 1;
        own = it.lds_rows + (b * kZrWaves + it.wave) * kSlotComps * RS;
        spare = it.lds_rows + ((b ^ 1) * kZrWaves + it.wave) * kSlotComps * RS;
        src_to_lds(it, own, ahead);
        // the block's edge rows come from memory; they are pushed after the
        // own row, which gives their loads time to land
        if constexpr (PK) {
            if (!it.share_m) load_row_pk(it, pk.vm, rm);
            if (!it.share_p) load_row_pk(it, pk.vp, rp);
        } else {
            if (!it.share_m) load_row(it, rm_, rm);
            if (!it.share_p) load_row(it, rp_, rp);
        }
        __syncthreads();
    } else if constexpr (ROLL) {
        ro = ahead;
        load_row(it, rm_, rm);
    } else {
        load_row(it, ro_, ro);
    }

    // Every schedule adds the rows in the same order -- own row, row y-1,
    // row y+1 -- so every tile forms each sum with the same roundings.
    // ---- own row: c_y = 0 directions and the rest population
    {
        Src s[PX];
        if constexpr (SHARE) {
            src_from_lds(it, own, s);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j) s[j] = make_src(ro.d[j], ro.vx[j], ro.vy[j], ro.vz[j]);
        }
        push_row<Q, 0, G, C, K, NL>(pl, s, zmask, it.ln);
        if (zmask & 2) {
            constexpr float w0 = (float)weight<Q>(0);
#pragma unroll
            for (int j = 0; j < PX; ++j) pl.c.v[0][j] = __builtin_fmaf(w0, s[j].a, pl.c.v[0][j]);
        }
    }
    // rolling prefetch: each row is requested one push ahead of its use, the
    // next plane's own row once this one's registers are free
    if constexpr (ROLL) load_row(it, rp_, rp);
    else if constexpr (!SHARE) load_row(it, rm_, rm);
    // shared rows: the next plane's own row, requested as soon as this
    // plane's own row has been pushed (its registers are free then; any
    // earlier and they would not fit), so its loads land during the rest of
    // the step.  Only where the instance has the registers for it at its
    // occupancy (EARLY_OK); D3Q27's larger sums keep the request at the end
    // of the step.
    constexpr bool EARLY = Q < 27 && EARLY_OK;
    if constexpr (EARLY) {
        if constexpr (PK) {
            chunk_voffs(it, tn_own, vn);
            load_row_pk(it, vn, ahead);
        } else if constexpr (SHARE) {
            load_row(it, wrapi((zs + 1) % nz, nz) * ny + it.yc, ahead);
        }
    }
    // ---- neighbour rows: y-1 sends its c_y = +1 directions, y+1 its c_y = -1
    {
        Src s[PX];
        if (SHARE && it.share_m) {
            src_from_lds(it, own - kSlotComps * RS, s);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j) s[j] = make_src(rm.d[j], rm.vx[j], rm.vy[j], rm.vz[j]);
        }
        push_row<Q, 1, G, C, K, NL>(pl, s, zmask, it.ln);
    }
    if constexpr (ROLL) load_row(it, wrapi((zs + 1) % nz, nz) * ny + it.yc, ahead);
    else if constexpr (!SHARE) load_row(it, rp_, rp);
    {
        Src s[PX];
        if (SHARE && it.share_p) {
            src_from_lds(it, own + kSlotComps * RS, s);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j) s[j] = make_src(rp.d[j], rp.vx[j], rp.vy[j], rp.vz[j]);
        }
        push_row<Q, -1, G, C, K, NL>(pl, s, zmask, it.ln);
    }
    // ---- halfway bounce-back at this plane's wall nodes (static list)
    if (zmask & 2)
        bounce_list<Q, P, G, C, K>(it, pl.c, wp, zc, wv, SHARE ? own : nullptr,
                                   SHARE ? spare : it.lds_res);
    wp.cur0 = wp.next0;
    wp.cur1 = wp.next1;
    wp.cur = e_next;
    wp.next0 = nn0;
    wp.next1 = nn1;

    // ---- plane zs - 1 is complete: finalise and store whole chunks, solid
    // slots included (they rewrite their zeros), so every line is written whole
    if ((zmask & 1) && it.active) {
        const int ro2 = (wrapi(zc - 1, nz) * ny + it.yc) * it.nx * ZrItem<P, G, C, K>::ES;
        const int so = G == 1 ? ro2 : 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float od[K], ox[K], oy[K], oz[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int sl = c * K + j;
                const bool f = (fluid_prev >> sl) & 1u;
                const float d = pl.m.v[0][sl];
                const float r = __builtin_amdgcn_rcpf(1.0f + d);
                od[j] = f ? d : 0.0f;
                ox[j] = f ? __builtin_fmaf(pl.m.v[1][sl], r, it.gx) : 0.0f;
                oy[j] = f ? __builtin_fmaf(pl.m.v[2][sl], r, it.gy) : 0.0f;
                oz[j] = f ? __builtin_fmaf(pl.m.v[3][sl], r, it.gz) : 0.0f;
            }
            const int vo = PK ? pk.vst[c] : it.voff[c] + (G == 1 ? 0 : ro2);
            if constexpr (PK) {
                // an all-solid chunk's offset stays out of range in every array
                // (unsigned 32-bit sums below 2^32: 4 * abytes <= kOob)
                const uint32_t u = (uint32_t)vo, ab = (uint32_t)it.abytes;
                store_chunk<P, K>(it.post[0], vo, 0, od, it.sr);
                store_chunk<P, K>(it.post[0], (int)(u + ab), 0, ox, it.su);
                store_chunk<P, K>(it.post[0], (int)(u + 2 * ab), 0, oy, it.su);
                store_chunk<P, K>(it.post[0], (int)(u + 3 * ab), 0, oz, it.su);
            } else {
                store_chunk<P, K>(it.post[0], vo, so, od, it.sr);
                store_chunk<P, K>(it.post[1], vo, so, ox, it.su);
                store_chunk<P, K>(it.post[2], vo, so, oy, it.su);
                store_chunk<P, K>(it.post[3], vo, so, oz, it.su);
            }
        }
    }
    fluid_prev = fown;
    if constexpr (!EARLY) {
        if constexpr (PK) {
            chunk_voffs(it, tn_own, vn);
            load_row_pk(it, vn, ahead);
        } else if constexpr (SHARE) {
            load_row(it, wrapi((zs + 1) % nz, nz) * ny + it.yc, ahead);
        }
    }
    if constexpr (PK) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            pk.vst[c] = pk.vcur[c];
            pk.vcur[c] = vn[c];
        }
        if (!it.share_m) chunk_voffs(it, tn_m, pk.vm);
        if (!it.share_p) chunk_voffs(it, tn_p, pk.vp);
    }
}

template <int PX>
__device__ __forceinline__ void zero_plane(Plane<PX>& q) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < PX; ++j) q.v[c][j] = 0.0f;
}

// One work item: G rows starting at row-group rg, destination planes [z0, z1).
// The three destination planes rotate roles statically (the march is
// unrolled by three), so no partial sums are copied between planes.
// The sample descriptor is read field by field with its own types and every
// value is marked wave-uniform, so per-item quantities live in scalar registers.
// EARLY_OK: the shared-row schedules request the next plane's own row right
// after this plane's own row is pushed.
template <int Q, int P, int G, int C, int K, int NL, int MODE, bool EARLY_OK>
__device__ __forceinline__ void zr_item(const StepArgs& a, const SampleDev* sd, int rg, int z0,
                                        int z1, float* __restrict__ lds, int wave,
                                        float* __restrict__ lds_rows) {
    using St = Storage<P>;
    using S = typename St::S;
    using It = ZrItem<P, G, C, K>;
    constexpr int PX = C * K;
    It it;
    it.lane = __lane_id();
    // with one row per wave the row is uniform; with G rows it depends on the lane group
    const int grp = G == 1 ? 0 : it.lane / It::Lg;
    it.gl = G == 1 ? it.lane : it.lane % It::Lg;
    // lanes L..63 of a one-row layout with idle lanes hold no nodes: their
    // offsets are out of range (no loads, no stores) and the lane moves skip
    // them (each keeps its own value)
    const bool idle = it.gl >= NL;
    it.ln.first = it.gl == 0 ? ~0u : 0u;
    it.ln.last = it.gl == NL - 1 ? ~0u : 0u;
    it.ln.up = (idle ? it.gl : (it.gl == 0 ? NL - 1 : it.gl - 1)) << 2;
    it.ln.down = (idle ? it.gl : (it.gl == NL - 1 ? 0 : it.gl + 1)) << 2;
    it.nx = __builtin_amdgcn_readfirstlane(sd->nx);
    it.ny = __builtin_amdgcn_readfirstlane(sd->ny);
    it.nz = __builtin_amdgcn_readfirstlane(sd->nz);
    it.xw = __builtin_amdgcn_readfirstlane(sd->xwords);
    it.z0 = z0; it.z1 = z1;
    const int y = rg * G + grp;
    it.active = y < it.ny;
    it.y0 = rg * G;
    it.yc = it.active ? y : it.ny - 1;
    it.ym = wrapi(it.yc - 1, it.ny);
    it.yp = wrapi(it.yc + 1, it.ny);
    const int64_t stride = uniform64(sd->stride);
    const uint32_t abytes = (uint32_t)(stride * It::ES);
    it.abytes = (int)abytes;
    const int64_t st0 = uniform64(sd->state[0]), st1 = uniform64(sd->state[1]);
    const S* pre = reinterpret_cast<const S*>(a.base + (a.parity ? st1 : st0));
    S* post = reinterpret_cast<S*>(a.base + (a.parity ? st0 : st1));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        it.pre[c] = make_rsrc(pre + c * stride, zr_packed(G, MODE) ? 4 * abytes : abytes);
        it.post[c] = make_rsrc(post + c * stride, zr_packed(G, MODE) ? 4 * abytes : abytes);
    }
    it.xm = make_rsrc(a.base + uniform64(sd->xmask),
                      (uint32_t)(((int64_t)it.xw * it.ny * it.nz + 2) * 4));
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int x0 = c * (NL * K) + it.gl * K;
        it.voff[c] = idle ? kOob : x0 * It::ES;
        it.woff[c] = idle ? 0 : (x0 >> 5) * 4;
        it.wsh[c] = idle ? 0 : x0 & 31;
    }
    it.isr = inv_scale_rho<P>(a); it.isu = inv_scale_u<P>(a);
    it.sr = scale_rho<P>(a); it.su = scale_u<P>(a);
    it.gx = 2.0f * a.ghf[0]; it.gy = 2.0f * a.ghf[1]; it.gz = 2.0f * a.ghf[2];
    it.woffs = (wofs_t*)(a.base + uniform64(sd->wall_off));
    it.wl = make_rsrc(a.base + uniform64(sd->wall_list),
                      (uint32_t)(uniform64(sd->n) * (int64_t)sizeof(typename WallEntry<Q>::type)));
    it.lds_res = lds;
    it.lds_rows = lds_rows;
    it.wave = wave;
    // rows y -/+ 1 are the neighbouring waves' rows: the block's waves hold
    // consecutive rows, and a row past ny wraps to a row outside the block
    it.share_m = wave > 0;
    it.share_p = wave < kZrWaves - 1 && y + 1 < it.ny;
    it.ctab = (ctab_t*)(a.base + uniform64(sd->chunk_tab));

    Plane<PX> A, B, Cp;
    zero_plane(A);
    zero_plane(B);
    zero_plane(Cp);
    uint32_t fluid_prev = 0;
    uint32_t win_next[C];
    load_windows(it, wrapi((z0 - 1) % it.nz, it.nz), win_next);
    WallPipe<Q> wp;
    wp.cur0 = wp.cur1 = 0;
    wp.cur = 0;
    wall_offsets(it, z0, wp.next0, wp.next1);
    // own row of the first source plane, requested ahead (shared rows and
    // rolling prefetch)
    RawRow<PX> rm;
    PkPipe<C> pk;
    if constexpr (zr_packed(G, MODE)) {
        const int zp = wrapi((z0 - 1) % it.nz, it.nz) * it.ny;
        RowTab<C> t;
        row_tab(it, zp + it.yc, t);
        chunk_voffs(it, t, pk.vcur);
#pragma unroll
        for (int c = 0; c < C; ++c) pk.vst[c] = kOob;  // plane z0 - 2 is not stored
        row_tab(it, zp + it.ym, t);
        chunk_voffs(it, t, pk.vm);
        row_tab(it, zp + it.yp, t);
        chunk_voffs(it, t, pk.vp);
        load_row_pk(it, pk.vcur, rm);
    } else if constexpr (MODE != 0) {
        load_row(it, wrapi((z0 - 1) % it.nz, it.nz) * it.ny + it.yc, rm);
    }
    int zs = z0 - 1;
    while (true) {
        zr_step<Q, P, G, C, K, NL, MODE, EARLY_OK>(it, zs, Planes<PX>{A, B, Cp}, win_next, fluid_prev, wp, rm, pk);
        zero_plane(A);
        if (++zs > z1) break;
        zr_step<Q, P, G, C, K, NL, MODE, EARLY_OK>(it, zs, Planes<PX>{B, Cp, A}, win_next, fluid_prev, wp, rm, pk);
        zero_plane(B);
        if (++zs > z1) break;
        zr_step<Q, P, G, C, K, NL, MODE, EARLY_OK>(it, zs, Planes<PX>{Cp, A, B}, win_next, fluid_prev, wp, rm, pk);
        zero_plane(Cp);
        if (++zs > z1) break;
    }
}

// The packed shared-row schedule (mode 3) of FP32 D3Q15 and D3Q19, per lane
// layout: the waves per SIMD its instance is built for -- the occupancy its
// registers and row slots give without the early request of the next
// plane's own row -- and whether it makes that request, which it does
// wherever the extra registers fit that occupancy without spilling (not at
// nx = 256: 4 waves and 128 registers leave no room).  +4 % on the 64-sample
// batch against the request for six or more nodes per lane only.  The other
// schedules, storage formats and lattices, where the same request would cost
// occupancy or spill in some layouts, keep that rule.  (The multi-row
// layouts have no shared-row schedule: 0 and false.)
constexpr int kShareWaves[kNumVariants] = {5, 5, 4, 4, 3, 2, 2, 0, 5, 3, 3, 2, 0, 0, 0};
constexpr bool kShareEarly[kNumVariants] = {true,  true, true,  false, true,  true,  true, false,
                                            true,  true, true,  true,  false, false, false};

constexpr bool zr_tabled(int q, int p, int mode) { return mode == 3 && p == kF32 && q < 27; }

// Whether instance (Q, P, V, MODE) requests the next plane's own row early.
constexpr bool zr_early(int q, int p, int v, int mode) {
    return zr_tabled(q, p, mode) ? kShareEarly[v] : kVariants[v].c * kVariants[v].k >= 6;
}

// Occupancy target of an instance: the tabled schedules at their layout's
// kShareWaves; the other shared-row schedules (one row per wave) and modes 1
// and 3 on the multi-row layouts at two waves per SIMD or more (at most 256
// registers per lane; the row slots of two workgroups fill a CU's LDS at the
// longest rows); the other instances at one or more.  Modes 1/3 and 2 are the
// same rolling-prefetch schedule on a multi-row layout, so the tile picks the
// occupancy there.
constexpr int zr_waves_per_simd(int q, int p, int v, int mode) {
    const int g = kVariants[v].g;
    if (zr_share(g, mode) && zr_tabled(q, p, mode)) return kShareWaves[v];
    return (zr_share(g, mode) || (g != 1 && (mode == 1 || mode == 3))) ? 2 : 1;
}

// Work item (4 x int32): sample, row group, z-segment start, z-segment end.
// Workgroups are remapped so that each XCD walks a contiguous range of items
// (neighbouring rows share their y-1 / y+1 reads in that XCD's L2).  Each
// instance compiles one lane layout V (its register budget alone sets the
// occupancy); batches of differently sized samples launch one instance per
// layout present.
template <int Q, int P, int V, int MODE>
__global__ __launch_bounds__(kZrThreads)
__attribute__((amdgpu_waves_per_eu(zr_waves_per_simd(Q, P, V, MODE))))
void k_zmarch(StepArgs a) {
    static_assert(V >= 0 && V < kNumVariants, "one lane layout per instance");
    constexpr int G = kVariants[V].g, C = kVariants[V].c, K = kVariants[V].k, NL = kVariants[V].l;
    static_assert(NL == 64 / G || (G == 1 && C == 1), "idle lanes only in one-chunk, one-row layouts");
    constexpr int kPX = C * K;
    constexpr bool kShare = zr_share(G, MODE);
    // shared rows: [2 planes][kZrWaves][kSlotComps][64 * kPX] (the bounce-back
    // sums use the other plane's slot); otherwise bounce-back sums
    // [kZrWaves][4][64 * kPX]
    constexpr int kLds = kShare ? 2 * kZrWaves * kSlotComps * kPX * 64 : kZrWaves * 4 * kPX * 64;
    __shared__ float lds_all[kLds];
    const int wave = threadIdx.x >> 6;
    float* lds_wave = lds_all + wave * 4 * kPX * 64;
    if constexpr (!kShare) {
        // bounce-back sums start at zero; every use clears what it read
        for (int i = __lane_id(); i < 4 * kPX * 64; i += 64) lds_wave[i] = 0.0f;
        __builtin_amdgcn_wave_barrier();
    }
    const int nwg = gridDim.x;
    const int b = blockIdx.x;
    // XCD-aware order: dispatch is round-robin over 8 XCDs
    const int per = (nwg + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int lb = xcd * per + k;
    const int nwaves = ((nwg + 7) / 8) * 8 * kZrWaves;
    // the item index is uniform across the wave; say so, so that every
    // per-item quantity (sample descriptor, buffer resources) stays scalar
    const int first = __builtin_amdgcn_readfirstlane(lb * kZrWaves + wave);
    for (int item = first; item < a.ntiles; item += nwaves) {
        // the work list is constant while a step runs: a scalar load
        typedef int wi4 __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(4))) wi4 item_t;
        const wi4 t = ((item_t*)a.tiles)[item];
        zr_item<Q, P, G, C, K, NL, MODE, zr_early(Q, P, V, MODE)>(a, a.samples + t.x, t.y, t.z,
                                                                 t.w, lds_wave, wave, lds_all);
    }
}

// Lane layouts of the one-launch kernel: one row per wave in one chunk (rows
// of 64-320 nodes).  The two-chunk rows (384, 512) would raise the kernel's
// register demand past the two-waves-per-SIMD budget; they launch alone.
constexpr bool zr_rows_layout(const ZrVariant& v) { return v.g == 1 && v.c == 1; }

// Widest row (nodes per lane) of those layouts.
constexpr int zr_rows_px() {
    int m = 0;
    for (int v = 0; v < kNumVariants; ++v)
        if (zr_rows_layout(kVariants[v]) && kVariants[v].k > m) m = kVariants[v].k;
    return m;
}

// Work item of lane layout v (dispatch of k_zmarch_rows): the arm of V == v
// runs it.
template <int Q, int P, int MODE, int V = 0>
__device__ __forceinline__ void zr_rows_item(const StepArgs& a, int v, int s, int rg, int z0,
                                             int z1, float* lds_all, int wave) {
    if constexpr (V < kNumVariants) {
        constexpr ZrVariant L = kVariants[V];
        if constexpr (zr_rows_layout(L)) {
            if (v == V) {
                // every layout requests the next plane's own row early: all
                // run at two waves per SIMD here (+5 % on the 64-sample batch)
                zr_item<Q, P, 1, 1, L.k, L.l, MODE, true>(a, a.samples + s, rg, z0, z1,
                                                    lds_all + wave * 4 * L.k * 64, wave, lds_all);
                return;
            }
        }
        zr_rows_item<Q, P, MODE, V + 1>(a, v, s, rg, z0, z1, lds_all, wave);
    }
}

// Every one-row, one-chunk lane layout in one launch (rows shared through
// LDS: mode 1 dense, mode 3 packed).  The work list is the concatenation of the layouts'
// lists, each in blocks of kZrWaves consecutive row items (one z-segment
// length per layout), so the four waves of a workgroup always take one block
// of one sample and run one layout's code; the item's sample names the
// layout.  The row slots are sized for the widest row, and the register
// budget is that of the widest layout, so every layout runs at two waves per
// SIMD.  The arithmetic is the per-layout kernel's, in the same order.
template <int Q, int P, int MODE>
__global__ __launch_bounds__(kZrThreads)
__attribute__((amdgpu_waves_per_eu(2)))
void k_zmarch_rows(StepArgs a) {
    static_assert(MODE == 1 || MODE == 3, "shared-row schedules only");
    constexpr int kLds = 2 * kZrWaves * kSlotComps * zr_rows_px() * 64;
    __shared__ float lds_all[kLds];
    const int wave = threadIdx.x >> 6;
    const int nwg = gridDim.x;
    const int b = blockIdx.x;
    const int per = (nwg + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int lb = xcd * per + k;
    const int nwaves = ((nwg + 7) / 8) * 8 * kZrWaves;
    const int first = __builtin_amdgcn_readfirstlane(lb * kZrWaves + wave);
    for (int item = first; item < a.ntiles; item += nwaves) {
        typedef int wi4 __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(4))) wi4 item_t;
        const wi4 t = ((item_t*)a.tiles)[item];
        const int v = __builtin_amdgcn_readfirstlane(a.samples[t.x].variant);
        zr_rows_item<Q, P, MODE>(a, v, t.x, t.y, t.z, t.w, lds_all, wave);
    }
}

// Kernel table of one (lattice, precision) pair; defined in the per-pair
// translation units built from tau1_zmarch_inst.hip (and, for the one-launch
// kernels of all one-row layouts, tau1_zmarch_rows.hip).
#define TAU1_ZM_TABLE_DECL(QQ, PP) \
    void* zm_kernel_##QQ##_##PP(int variant, int mode); void* ck_kernel_##QQ##_##PP(int k); \
    void* zr_rows_kernel_##QQ##_##PP(int mode);
TAU1_ZM_TABLE_DECL(15, 1) TAU1_ZM_TABLE_DECL(15, 2) TAU1_ZM_TABLE_DECL(15, 3)
TAU1_ZM_TABLE_DECL(19, 1) TAU1_ZM_TABLE_DECL(19, 2) TAU1_ZM_TABLE_DECL(19, 3)
TAU1_ZM_TABLE_DECL(27, 1) TAU1_ZM_TABLE_DECL(27, 2) TAU1_ZM_TABLE_DECL(27, 3)
#undef TAU1_ZM_TABLE_DECL

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
inline int zr_xwords(int nx) { return (nx + 2 + 31) / 32 + 1; }

inline bool zmarch_precision_ok(int prec) { return prec == kF32 || prec == kF16 || prec == kBF16; }

// Tiles of a context: modes 0-2 on the dense layout, mode 3 and the chunk
// tile on the packed layout.
inline bool zmarch_tile_ok(int prec, bool packed, int tile) {
    return zmarch_precision_ok(prec) && tile >= 0 && tile < kNumTiles &&
           tile_packed(tile) == packed;
}

// z-segments of 64 planes
inline int zmarch_default_tile(bool packed) { return packed ? 14 : 2; }

inline void* pick_zmarch(int q, int p, int variant, int mode) {
    switch (q * 10 + p) {
        case 151: return zm_kernel_15_1(variant, mode);
        case 152: return zm_kernel_15_2(variant, mode);
        case 153: return zm_kernel_15_3(variant, mode);
        case 191: return zm_kernel_19_1(variant, mode);
        case 192: return zm_kernel_19_2(variant, mode);
        case 193: return zm_kernel_19_3(variant, mode);
        case 271: return zm_kernel_27_1(variant, mode);
        case 272: return zm_kernel_27_2(variant, mode);
        case 273: return zm_kernel_27_3(variant, mode);
    }
    return nullptr;
}

inline void* pick_chunks(int q, int p, int k) {
    switch (q * 10 + p) {
        case 151: return ck_kernel_15_1(k);
        case 152: return ck_kernel_15_2(k);
        case 153: return ck_kernel_15_3(k);
        case 191: return ck_kernel_19_1(k);
        case 192: return ck_kernel_19_2(k);
        case 193: return ck_kernel_19_3(k);
        case 271: return ck_kernel_27_1(k);
        case 272: return ck_kernel_27_2(k);
        case 273: return ck_kernel_27_3(k);
    }
    return nullptr;
}

inline void* pick_zmarch_rows(int q, int p, int mode) {
    switch (q * 10 + p) {
        case 151: return zr_rows_kernel_15_1(mode);
        case 152: return zr_rows_kernel_15_2(mode);
        case 153: return zr_rows_kernel_15_3(mode);
        case 191: return zr_rows_kernel_19_1(mode);
        case 192: return zr_rows_kernel_19_2(mode);
        case 193: return zr_rows_kernel_19_3(mode);
        case 271: return zr_rows_kernel_27_1(mode);
        case 272: return zr_rows_kernel_27_2(mode);
        case 273: return zr_rows_kernel_27_3(mode);
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

// Supported when every sample has a lane layout and each state array and
// mask fits the 32-bit buffer offsets below the out-of-range offset.
template <typename SH>
inline bool zmarch_supported(int q, int prec, const SH* s, int n) {
    if (!zmarch_precision_ok(prec)) return false;
    const int64_t es = storage_bytes(prec);
    for (int i = 0; i < n; ++i) {
        const SampleDev& sd = s[i].dev;
        if (sd.variant < 0) return false;
        if (sd.stride * es + 65536 > (int64_t)kOob) return false;
        if (((int64_t)sd.xwords * sd.ny * sd.nz + 2) * 4 + 65536 > (int64_t)kOob) return false;
        if (sd.n * (q > 19 ? 8 : 4) + 65536 > (int64_t)kOob) return false;  // wall list
    }
    return true;
}

inline void zmarch_tiling(SampleDev& sd) {
    sd.variant = zr_variant_for(sd.nx);
    sd.xwords = zr_xwords(sd.nx);
    const int g = sd.variant >= 0 ? kVariants[sd.variant].g : 1;
    sd.tiles_y = (sd.ny + g - 1) / g;
}

// Row groups of a sample in the work list: with shared rows (one row per
// wave, `blocks`), padded to whole blocks of kZrWaves rows, so that the waves
// of a workgroup always hold one block of consecutive rows with the same
// z-segment (the extra rows are inactive: they store nothing).
inline int zmarch_rows(const SampleDev& sd, bool blocks) {
    if (blocks && sd.variant >= 0 && kVariants[sd.variant].g == 1)
        return (sd.tiles_y + kZrWaves - 1) / kZrWaves * kZrWaves;
    return sd.tiles_y;
}

// Work list of the samples with lane layout `variant`, for z-segment length
// lz: items (sample, row group, z0, z1) with row groups fastest so
// neighbouring rows are neighbouring items.  Only items with a fluid node in
// their rows and planes are listed (`s[i].rowfluid`, one flag per row
// y + ny z, when present): the others would store nothing, and their rows'
// state is read from memory by the items next to them.  With shared rows
// (`blocks`) a block of kZrWaves row items is kept or dropped as a whole, so
// the waves of a workgroup still march the same z-segment.
template <typename SH>
inline std::vector<int32_t> zmarch_worklist(const SH* s, int n, int lz, int variant, bool blocks) {
    std::vector<int32_t> out;
    for (int i = 0; i < n; ++i) {
        const SampleDev& sd = s[i].dev;
        if (sd.variant < 0 || sd.variant != variant) continue;
        const int rows = zmarch_rows(sd, blocks);
        const int g = kVariants[sd.variant].g;
        const int step = blocks && g == 1 ? kZrWaves : 1;  // row items kept together
        const auto& rf = s[i].rowfluid;
        for (int z0 = 0; z0 < sd.nz; z0 += lz) {
            const int z1 = z0 + lz < sd.nz ? z0 + lz : sd.nz;
            for (int rg0 = 0; rg0 < rows; rg0 += step) {
                bool busy = rf.empty();
                const int y0 = rg0 * g, y1 = std::min((rg0 + step) * g, sd.ny);
                for (int z = z0; z < z1 && !busy; ++z)
                    for (int y = y0; y < y1 && !busy; ++y) busy = rf[(size_t)z * sd.ny + y] != 0;
                if (!busy) continue;
                for (int rg = rg0; rg < rg0 + step; ++rg) {
                    out.push_back(i);
                    out.push_back(rg);
                    out.push_back(z0);
                    out.push_back(z1);
                }
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
        items += (int64_t)zmarch_rows(sd, true) * ((sd.nz + tile_lz(0) - 1) / tile_lz(0));
    }
    return items;
}

// Autotune cache: one line per entry "tau1 <arch> q<Q> p<P> n<bucket> tile <t> ms <x>".
inline int64_t size_bucket(int64_t n) {
    int64_t b = 1;
    while (b < n) b <<= 1;
    return b;
}

inline int zmarch_cache_lookup(const char* path, int q, int p, int64_t nodes, bool packed) {
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
            std::strcmp(arch, "gfx950") == 0 && qq == q && pp == p && nb == bucket &&
            zmarch_tile_ok(p, packed, tile))
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
