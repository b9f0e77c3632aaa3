// tau1_chunks.hpp -- step kernel over the stored chunks of the packed layout.
//
// In a porous medium of low porosity most lane chunks of a row are solid, yet
// the z-march evaluates every node of every row segment that holds fluid.
// This kernel's work follows the stored chunks instead: one lane per chunk of
// the packed layout (K consecutive x-nodes holding at least one fluid node),
// 64 consecutive chunks of one sample per wave, in storage order, so the
// lane's own chunk is read and written with coalesced vector accesses.
//
// For each of its K nodes the lane gathers the equilibria of Eq. (3) that the
// neighbours send it (the pull form of Eqs. (9)-(10)): it reads the nine
// (y, z) neighbour columns of its chunk -- the chunk at the same x-position
// in each neighbour row, plus the node on either side in x where a direction
// needs it -- at the packed positions that the chunk's nine neighbour-row
// records give (built once from the chunk table, so a step reads the state
// one dependent load after the records), and an all-solid chunk reads as
// zeros, which a solid node sends anyway.  Halfway bounce-back (Eq. 11)
// returns the node's own equilibria along its solid links, which come from
// the extended solid mask of the same nine rows.
//
// Every destination sum is formed in the order in which the z-march forms
// it: source plane z-1, then z, then z+1; within a plane the own row, then
// row y-1, then row y+1; within a row the lattice directions in order; the
// rest population after the own row of plane z and the wall returns after
// row y+1 of plane z.  Both kernels therefore give the same bits, and the
// autotuner may pick either.
#pragma once

#include "tau1_zmarch.hpp"

namespace tau1 {

template <int Q, int CY, int CZ, int KD = 1>
constexpr bool ck_has_dir() {
    if constexpr (KD >= Q) {
        return false;
    } else {
        using L = Lattice<Q>;
        return (L::c[KD].y == CY && L::c[KD].z == CZ) || ck_has_dir<Q, CY, CZ, KD + 1>();
    }
}

// Whether some direction of the column (c_y, c_z) = (CY, CZ) has c_x != 0:
// its sources then include the nodes on either side of the chunk.
template <int Q, int CY, int CZ, int KD = 1>
constexpr bool ck_needs_edges() {
    if constexpr (KD >= Q) {
        return false;
    } else {
        using L = Lattice<Q>;
        return (L::c[KD].y == CY && L::c[KD].z == CZ && L::c[KD].x != 0) ||
               ck_needs_edges<Q, CY, CZ, KD + 1>();
    }
}

struct CkCtx {
    rsrc_t pre, post;         // the read and the written buffer (four arrays each)
    int abytes;               // bytes per array
    const uint32_t* xm;       // extended solid mask
    int nx, ny, nz, xw, nch;  // nch: chunks per row
    float isr, isu;
};

// Lane moves across the whole wave: from lane l - 1 (ror) and from lane l + 1
// (rol).  Every lane has a source, so no previous value is needed.
__device__ __forceinline__ float ck_from_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x13C, 0xf, 0xf, true));  // wave_ror:1
}
__device__ __forceinline__ float ck_from_next(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x134, 0xf, 0xf, true));  // wave_rol:1
}

// Where a lane's x-neighbour chunks are: the lanes before and after it hold
// the chunks ci - 1 and ci + 1 of the same row when those are stored (the
// list is in storage order); otherwise the edge node is read from memory.
struct CkNb {
    bool left, right;  // lane l - 1 / l + 1 holds chunk ci - 1 / ci + 1 of this row
    int cl, cr;        // the neighbour chunk indices (periodic in x)
};

// Source terms of the column's nodes x0 - 1 .. x0 + K (slots 0 .. K + 1); the
// two edge slots only where a direction of the column needs them.  Every
// lane of the wave takes part (the edge values move between lanes).  All
// reads of a column are addressed from its record alone, so they are in
// flight together; the edge reads of lanes whose neighbour lane holds the
// edge use an out-of-range offset (no memory access) instead of a branch.
template <int P, int K, bool EDGES>
__device__ __forceinline__ void ck_column(const CkCtx& c, const ck_rec_t& rec, int ci,
                                          const CkNb& nb, Src (&s)[K + 2]) {
    constexpr int ES = (int)sizeof(typename Storage<P>::S);
    constexpr uint32_t CB = (uint32_t)(K * ES);
    const uint32_t rank = rec.x & kRecIndex;
    const uint32_t sc = (rec.x >> 30) & 1u;
    const int vo = sc ? (int)(rank * CB) : kOob;
    float v[4][K];
    load_chunk<P, K>(c.pre, vo, 0, v[0], c.isr);
    load_chunk<P, K>(c.pre, vo, c.abytes, v[1], c.isu);
    load_chunk<P, K>(c.pre, vo, 2 * c.abytes, v[2], c.isu);
    load_chunk<P, K>(c.pre, vo, 3 * c.abytes, v[3], c.isu);
    float e[2][4];
    if constexpr (EDGES) {
        // chunk ci - 1 is the stored chunk before position ci, chunk ci + 1 the
        // one after chunk ci; across the periodic x boundary the record names it
        const uint32_t wrap = rec.y & kRecIndex;
        const bool wok = (rec.y >> 31) != 0u;
        int ol, orr;
        if (ci > 0) ol = ((rec.x >> 29) & 1u) ? (int)((rank - 1u) * CB) : kOob;
        else ol = wok ? (int)(wrap * CB) : kOob;
        if (ci + 1 < c.nch) orr = (rec.x >> 31) ? (int)((rank + sc) * CB) : kOob;
        else orr = wok ? (int)(wrap * CB) : kOob;
        ol = (nb.left || ol == kOob) ? kOob : ol + (K - 1) * ES;
        orr = nb.right ? kOob : orr;
        e[0][0] = load_one<P>(c.pre, ol, 0, c.isr);
        e[1][0] = load_one<P>(c.pre, orr, 0, c.isr);
#pragma unroll
        for (int a = 1; a < 4; ++a) {
            e[0][a] = load_one<P>(c.pre, ol, a * c.abytes, c.isu);
            e[1][a] = load_one<P>(c.pre, orr, a * c.abytes, c.isu);
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) s[j + 1] = make_src(v[0][j], v[1][j], v[2][j], v[3][j]);
    if constexpr (EDGES) {
        // last node of the chunk before, first node of the chunk after: from
        // the neighbouring lanes' loads of this column where they hold those
        // chunks
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const float pv = ck_from_prev(v[a][K - 1]);
            const float nv = ck_from_next(v[a][0]);
            e[0][a] = nb.left ? pv : e[0][a];
            e[1][a] = nb.right ? nv : e[1][a];
        }
        s[0] = make_src(e[0][0], e[0][1], e[0][2], e[0][3]);
        s[K + 1] = make_src(e[1][0], e[1][1], e[1][2], e[1][3]);
    }
}

// Adds the contributions of one source column: every direction k with
// (c_y, c_z) = (CY, CZ), in order, from source node x - c_x to node x.  The
// multiply-adds are those of the z-march's push (add_to).
template <int Q, int CY, int CZ, int K, int KD = 1>
__device__ __forceinline__ void ck_pull(float (&acc)[4][K], const Src (&s)[K + 2]) {
    if constexpr (KD < Q) {
        using L = Lattice<Q>;
        constexpr int CX = L::c[KD].x;
        if constexpr (L::c[KD].y == CY && L::c[KD].z == CZ) {
            constexpr float w = (float)weight<Q>(KD);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const float u = feq_m<CX, CY, CZ>(s[j + 1 - CX]);
                acc[0][j] = __builtin_fmaf(w, u, acc[0][j]);
                if constexpr (CX != 0) acc[1][j] = __builtin_fmaf(CX * w, u, acc[1][j]);
                if constexpr (CY != 0) acc[2][j] = __builtin_fmaf(CY * w, u, acc[2][j]);
                if constexpr (CZ != 0) acc[3][j] = __builtin_fmaf(CZ * w, u, acc[3][j]);
            }
        }
        ck_pull<Q, CY, CZ, K, KD + 1>(acc, s);
    }
}

// Source column (source row offset -CY, plane offset -CZ from the node): its
// directions c_y = CY, c_z = CZ.
template <int Q, int P, int CY, int CZ, int K>
__device__ __forceinline__ void ck_source(const CkCtx& c, const ck_rec_t (&rec)[9], int ci,
                                          const CkNb& nb, float (&acc)[4][K]) {
    if constexpr (ck_has_dir<Q, CY, CZ>()) {
        Src s[K + 2];
        ck_column<P, K, ck_needs_edges<Q, CY, CZ>()>(c, rec[(1 - CY) * 3 + 1 - CZ], ci, nb, s);
        ck_pull<Q, CY, CZ, K>(acc, s);
    }
}

// Solid neighbours per direction: bit j of m[k] is set when node x0 + j + c_k
// is solid, from the nine mask windows win[CY + 1][CZ + 1] (bit b: node
// x0 - 1 + b).  One shift per direction serves all K nodes of the chunk.
template <int Q, int KD = 1>
__device__ __forceinline__ void ck_solid_dirs(const uint32_t (&win)[3][3], uint32_t (&m)[Q]) {
    if constexpr (KD < Q) {
        using L = Lattice<Q>;
        constexpr int CX = L::c[KD].x, CY = L::c[KD].y, CZ = L::c[KD].z;
        m[KD] = win[CY + 1][CZ + 1] >> (1 + CX);
        ck_solid_dirs<Q, KD + 1>(win, m);
    }
}

// Occupancy target by chunk length (the register need grows with it: every
// wave keeps the loads of several neighbour columns in flight): four waves
// per SIMD for one node, three for two, two for longer chunks.
constexpr int ck_waves_per_simd(int k) { return k == 1 ? 4 : k == 2 ? 3 : 2; }

template <int Q, int P, int K>
__global__ __launch_bounds__(kCkThreads)
__attribute__((amdgpu_waves_per_eu(ck_waves_per_simd(K))))
void k_chunks(StepArgs a) {
    using St = Storage<P>;
    constexpr int ES = (int)sizeof(typename St::S);
    const int wave = threadIdx.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kCkWaves + wave);
    if (item >= a.ntiles) return;
    typedef int wi4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(4))) wi4 item_t;
    const wi4 t = ((item_t*)a.tiles)[item];
    // lanes past the item's chunks repeat the first chunk and store nothing
    // (all lanes stay active: edge values move between lanes)
    const int lane = __lane_id();
    const bool valid = lane < t.z;
    const SampleDev* sd = a.samples + t.x;

    CkCtx c;
    c.nx = __builtin_amdgcn_readfirstlane(sd->nx);
    c.ny = __builtin_amdgcn_readfirstlane(sd->ny);
    c.nz = __builtin_amdgcn_readfirstlane(sd->nz);
    c.xw = __builtin_amdgcn_readfirstlane(sd->xwords);
    c.nch = c.nx / K;
    const int64_t stride = uniform64(sd->stride);
    c.abytes = (int)(uint32_t)(stride * ES);
    const int64_t st0 = uniform64(sd->state[0]), st1 = uniform64(sd->state[1]);
    c.pre = make_rsrc(a.base + (a.parity ? st1 : st0), 4u * (uint32_t)c.abytes);
    c.post = make_rsrc(a.base + (a.parity ? st0 : st1), 4u * (uint32_t)c.abytes);
    c.xm = reinterpret_cast<const uint32_t*>(a.base + uniform64(sd->xmask));
    c.isr = inv_scale_rho<P>(a);
    c.isu = inv_scale_u<P>(a);

    const int p = t.y + (valid ? lane : 0);  // packed index of the lane's chunk
    const uint32_t e = reinterpret_cast<const uint32_t*>(a.base + uniform64(sd->chunk_list))[p];
    // neighbour-row records: record (dy + 1) * 3 + dz + 1 for row (y + dy, z + dz)
    ck_rec_t rec[9];
    {
        const ck_rec_t* rb = reinterpret_cast<const ck_rec_t*>(a.base + uniform64(sd->chunk_nbr));
        const int64_t nchunks = uniform64(sd->nchunks);
#pragma unroll
        for (int i = 0; i < 9; ++i) rec[i] = rb[(int64_t)i * nchunks + p];
    }
    const int row = (int)(e >> kChunkBits), ci = (int)(e & ((1u << kChunkBits) - 1u));
    const int y = row % c.ny, z = row / c.ny;
    const int x0 = ci * K;
    // list entries grow with the packed index, so lane l - 1 holds chunk
    // ci - 1 of the same row exactly when its entry is e - 1 (and ci > 0)
    CkNb nb;
    {
        const int ei = (int)e;
        const int ep = __builtin_amdgcn_mov_dpp(ei, 0x13C, 0xf, 0xf, true);
        const int en = __builtin_amdgcn_mov_dpp(ei, 0x134, 0xf, 0xf, true);
        nb.left = lane > 0 && valid && ci > 0 && ep == ei - 1;
        nb.right = lane + 1 < t.z && ci + 1 < c.nch && en == ei + 1;
        nb.cl = ci == 0 ? c.nch - 1 : ci - 1;
        nb.cr = ci == c.nch - 1 ? 0 : ci + 1;
    }

    // solid windows of the nine neighbour rows: bit b is node x0 - 1 + b
    uint32_t win[3][3];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
            win[dy + 1][dz + 1] = xmask_window(
                c.xm, (int64_t)wrapi(z + dz, c.nz) * c.ny + wrapi(y + dy, c.ny), c.xw, x0);

    float acc[4][K];
#pragma unroll
    for (int comp = 0; comp < 4; ++comp)
#pragma unroll
        for (int j = 0; j < K; ++j) acc[comp][j] = 0.0f;

    // source plane z - 1 (directions with c_z = +1): own row, row y-1, row y+1
    ck_source<Q, P, 0, 1, K>(c, rec, ci, nb, acc);
    ck_source<Q, P, 1, 1, K>(c, rec, ci, nb, acc);
    ck_source<Q, P, -1, 1, K>(c, rec, ci, nb, acc);
    // source plane z: own row (c_y = c_z = 0), the rest population, rows y-1, y+1
    Src own[K + 2];
    ck_column<P, K, true>(c, rec[4], ci, nb, own);
    ck_pull<Q, 0, 0, K>(acc, own);
    {
        constexpr float w0 = (float)weight<Q>(0);
#pragma unroll
        for (int j = 0; j < K; ++j) acc[0][j] = __builtin_fmaf(w0, own[j + 1].a, acc[0][j]);
    }
    ck_source<Q, P, 1, 0, K>(c, rec, ci, nb, acc);
    ck_source<Q, P, -1, 0, K>(c, rec, ci, nb, acc);
    // wall returns of the fluid nodes with a solid link (for the others the
    // z-march adds zeros, which leaves the sums as they are)
    uint32_t sdir[Q];
    sdir[0] = 0u;
    ck_solid_dirs<Q>(win, sdir);
    uint32_t any = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) any |= sdir[k];
    const uint32_t fluid = ~(win[1][1] >> 1) & ((1u << K) - 1u);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if ((fluid & any) >> j & 1u) {
            float r[4];
            wall_sums<Q>(own[j + 1],
                         [&](int k) { return (uint32_t)__builtin_amdgcn_sbfe((int)sdir[k], j, 1); }, r);
#pragma unroll
            for (int comp = 0; comp < 4; ++comp) acc[comp][j] += r[comp];
        }
    }
    // source plane z + 1 (directions with c_z = -1)
    ck_source<Q, P, 0, -1, K>(c, rec, ci, nb, acc);
    ck_source<Q, P, 1, -1, K>(c, rec, ci, nb, acc);
    ck_source<Q, P, -1, -1, K>(c, rec, ci, nb, acc);

    // finalise (as the z-march) and store the chunk, solid slots as zeros
    const float gx = 2.0f * a.ghf[0], gy = 2.0f * a.ghf[1], gz = 2.0f * a.ghf[2];
    float od[K], ox[K], oy[K], oz[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool f = (fluid >> j) & 1u;
        const float d = acc[0][j];
        const float r = __builtin_amdgcn_rcpf(1.0f + d);
        od[j] = f ? d : 0.0f;
        ox[j] = f ? __builtin_fmaf(acc[1][j], r, gx) : 0.0f;
        oy[j] = f ? __builtin_fmaf(acc[2][j], r, gy) : 0.0f;
        oz[j] = f ? __builtin_fmaf(acc[3][j], r, gz) : 0.0f;
    }
    const float sr = scale_rho<P>(a), su = scale_u<P>(a);
    // a lane past the item's chunks stores out of range (dropped)
    const uint32_t vo = valid ? (uint32_t)p * (uint32_t)(K * ES) : (uint32_t)kOob;
    const uint32_t ab = (uint32_t)c.abytes;
    store_chunk<P, K>(c.post, (int)vo, 0, od, sr);
    store_chunk<P, K>(c.post, (int)(vo + ab), 0, ox, su);
    store_chunk<P, K>(c.post, (int)(vo + 2 * ab), 0, oy, su);
    store_chunk<P, K>(c.post, (int)(vo + 3 * ab), 0, oz, su);
}

}  // namespace tau1
