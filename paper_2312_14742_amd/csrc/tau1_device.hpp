// tau1_device.hpp -- device-side building blocks of the Tau1 step on gfx950:
// lattice tables, storage codecs and the per-sample descriptor the kernels read.
//
// Lattices: the DdQq sets named in the paper's complexity table (D3Q15, D3Q19,
// D3Q27) with the textbook weights of Qian, d'Humieres and Lallemand; c_s^2 =
// 1/3 so Eq. (3) carries the constants 3, 9/2 and 3/2.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

namespace tau1 {

// ---------------------------------------------------------------------------
// Direction sets.  Order: rest, six faces (+x -x +y -y +z -z), then edges and
// corners as opposite pairs, so that opp(k) = k+1 (k odd), k-1 (k even > 0).
// ---------------------------------------------------------------------------
struct Dir {
    int x, y, z;
};

template <int Q> struct Lattice;

template <> struct Lattice<19> {
    static constexpr int q = 19;
    static constexpr Dir c[19] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr double w_rest = 1.0 / 3.0, w_face = 1.0 / 18.0,
                            w_edge = 1.0 / 36.0, w_corner = 0.0;
};

template <> struct Lattice<15> {
    static constexpr int q = 15;
    static constexpr Dir c[15] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    static constexpr double w_rest = 2.0 / 9.0, w_face = 1.0 / 9.0,
                            w_edge = 0.0, w_corner = 1.0 / 72.0;
};

template <> struct Lattice<27> {
    static constexpr int q = 27;
    static constexpr Dir c[27] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    static constexpr double w_rest = 8.0 / 27.0, w_face = 2.0 / 27.0,
                            w_edge = 1.0 / 54.0, w_corner = 1.0 / 216.0;
};

// D2Q9, the two-dimensional lattice of the paper's validation runs (z = 0):
// rest, faces, then the diagonals as opposite pairs, as above.
template <> struct Lattice<9> {
    static constexpr int q = 9;
    static constexpr Dir c[9] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    static constexpr double w_rest = 4.0 / 9.0, w_face = 1.0 / 9.0,
                            w_edge = 1.0 / 36.0, w_corner = 0.0;
};

// Weight of a direction from its number of nonzero components.
template <int Q>
__host__ __device__ constexpr double weight(int k) {
    using L = Lattice<Q>;
    const int n = (L::c[k].x != 0) + (L::c[k].y != 0) + (L::c[k].z != 0);
    return n == 0 ? L::w_rest : n == 1 ? L::w_face : n == 2 ? L::w_edge : L::w_corner;
}

// ---------------------------------------------------------------------------
// Storage codecs.  The stored state per node is (drho, v) with drho = rho - 1
// and v = u + g/2 (the velocity the equilibrium is evaluated at).  Solid nodes
// hold exact zeros, so as sources they contribute nothing.
// ---------------------------------------------------------------------------
enum Precision : int { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

template <int P> struct Storage;
template <> struct Storage<kF64> {
    using S = double;
    using T = double;  // compute type
    static __device__ __forceinline__ T load(const S* p, int64_t i, T) { return p[i]; }
    static __device__ __forceinline__ void store(S* p, int64_t i, T v, T) { p[i] = v; }
};
template <> struct Storage<kF32> {
    using S = float;
    using T = float;
    static __device__ __forceinline__ T load(const S* p, int64_t i, T) { return p[i]; }
    static __device__ __forceinline__ void store(S* p, int64_t i, T v, T) { p[i] = v; }
};
// IEEE half with a power-of-two scale: stored = value * 2^s.  The scale keeps
// rho - 1 (~1e-7..1e-4) and u out of the half subnormal range.
template <> struct Storage<kF16> {
    using S = __half;
    using T = float;
    static __device__ __forceinline__ T load(const S* p, int64_t i, T inv_scale) {
        return __half2float(p[i]) * inv_scale;
    }
    static __device__ __forceinline__ void store(S* p, int64_t i, T v, T scale) {
        p[i] = __float2half_rn(v * scale);
    }
};
template <> struct Storage<kBF16> {
    using S = __hip_bfloat16;
    using T = float;
    static __device__ __forceinline__ T load(const S* p, int64_t i, T) {
        return __bfloat162float(p[i]);
    }
    static __device__ __forceinline__ void store(S* p, int64_t i, T v, T) {
        p[i] = __float2bfloat16(v);
    }
};

inline constexpr int storage_bytes(int prec) {
    return prec == kF64 ? 8 : prec == kF32 ? 4 : 2;
}

// ---------------------------------------------------------------------------
// Per-sample descriptor in device memory.  All offsets are byte offsets from
// the workspace base.  State buffer b (0 or 1) holds four arrays of `stride`
// elements: drho | vx | vy | vz.
//
// Two layouts of those arrays:
//   dense   element i is node i = x + nx (y + ny z);
//   packed  the nodes are cut into chunks of pk consecutive x-nodes (the
//           z-march lane chunks) and only chunks holding at least one fluid
//           node are stored, in node order; chunk table entry (row, c), rows
//           r = y + ny z, describes the 64 chunks c * 64 .. c * 64 + 63 of the
//           row: a 64-bit fluid bitmap (uint32 lo, hi) and the packed index of
//           its first fluid chunk (uint32), then one unused word.
// ---------------------------------------------------------------------------
// Wall-list entry: x (bits 0-9), y mod G (10-11), solid-neighbour bit of
// direction k at bit 11 + k.
template <int Q>
struct WallEntry {
    using type = typename std::conditional<(Q > 19), uint64_t, uint32_t>::type;
};

struct SampleDev {
    int64_t n;            // nodes
    int64_t stride;       // elements between the four state arrays
    int64_t state[2];     // byte offsets of buffer 0 and buffer 1
    int64_t mask;         // byte offset of the bit mask (uint32 words)
    int64_t block0;       // first block of this sample in a per-node launch
    int64_t xmask;        // byte offset of the extended (periodic) row mask
    int64_t wall_off;     // byte offset of the wall-list row offsets (uint32, rows + 1)
    int64_t wall_list;    // byte offset of the wall-list entries (one per wall node)
    int64_t chunk_tab;    // byte offset of the chunk table (packed layout)
    int64_t chunk_list;   // byte offset of the chunk list (packed layout, where the
                          // chunk tile may run; else 0): per stored chunk, in
                          // storage order, row y + ny z (bits 7..31) and chunk
                          // index in the row (bits 0..6)
    int64_t chunk_nbr;    // byte offset of the chunks' neighbour-row records (with
                          // the chunk list; else 0): 9 arrays, one per (y, z)
                          // neighbour row, of one uint2 per stored chunk
    int64_t nchunks;      // packed layout: stored chunks
    int64_t types;        // D2Q9: byte offset of the node types (uint8: 0 fluid,
                          // 1 wall, 2 moving wall); 0 otherwise
    int32_t nx, ny, nz;
    int32_t words;        // mask words per (y, z) row: ceil(nx / 32)
    int32_t xwords;       // extended-mask words per row
    int32_t variant;      // z-march lane layout (-1: not supported)
    int32_t tiles_y;      // z-march row groups
    int32_t pk;           // packed layout: nodes per chunk; 0 = dense layout
};

// Solid bit of node (x, y, z).
__device__ __forceinline__ uint32_t solid_bit(const uint32_t* mask, int words,
                                              int ny, int x, int y, int z) {
    const uint32_t w = mask[((int64_t)z * ny + y) * words + (x >> 5)];
    return (w >> (x & 31)) & 1u;
}

// Element index of node (x, y, z) (node index i) in the state arrays, or -1
// when the packed layout stores no chunk for it (its chunk is all solid).
__device__ __forceinline__ int64_t state_slot(const uint8_t* base, const SampleDev& sd, int x,
                                              int y, int z, int64_t i) {
    if (sd.pk == 0) return i;
    const int ci = x / sd.pk;
    const int groups = (sd.nx + 64 * sd.pk - 1) / (64 * sd.pk);  // a last group may be partial
    const uint4 e = reinterpret_cast<const uint4*>(base + sd.chunk_tab)
        [((int64_t)z * sd.ny + y) * groups + (ci >> 6)];
    const uint64_t bits = ((uint64_t)e.y << 32) | e.x;
    const int l = ci & 63;
    if (!((bits >> l) & 1u)) return -1;
    const uint64_t below = bits & ((uint64_t(1) << l) - 1u);
    return ((int64_t)e.z + __popcll(below)) * sd.pk + (x - ci * sd.pk);
}

}  // namespace tau1
