// tau1_service.hpp -- non-template service kernels (geometry encode, final
// reduction pass, copy probe).  Included by the host API translation unit only.
#pragma once

#include "tau1_kernels.hpp"

namespace tau1 {

// ---------------------------------------------------------------------------
// Geometry encode (a0): pack solid bytes of rows [row0, row0 + nrows) into
// 32-node words; one thread per word.  Rows are (y, z) pairs, row = y + ny z.
// ---------------------------------------------------------------------------
__global__ void k_pack_mask(const uint8_t* __restrict__ solid, uint32_t* __restrict__ mask,
                            int nx, int words, int64_t row0, int64_t nrows) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * words) return;
    const int64_t r = t / words;
    const int w = (int)(t % words);
    const uint8_t* src = solid + r * nx;
    uint32_t bits = 0;
    const int x0 = w * 32;
    const int x1 = min(x0 + 32, nx);
    for (int x = x0; x < x1; ++x) bits |= (src[x] != 0 ? 1u : 0u) << (x - x0);
    mask[(row0 + r) * words + w] = bits;
}

// Final pass over the kReduceBlocks partials (one block; thread t adds
// partials t, t + 256, ... in order, then the fixed wave butterfly and wave
// order of block_sum4); writes out[0] = mass, out[1] = permeability (or 0
// when g_axis == 0), out[2] = fluid count, out[3] = non-finite count.
__global__ __launch_bounds__(kReduceThreads) void k_reduce_final(const double* __restrict__ partial,
                                                                 int64_t n, double g_axis,
                                                                 double* __restrict__ out) {
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < kReduceBlocks; b += kReduceThreads)
        for (int c = 0; c < 4; ++c) acc[c] += partial[b * 4 + c];
    block_sum4(acc);
    if (threadIdx.x == 0) {
        const double sum_drho = acc[0], sum_u = acc[1], nf = acc[2];
        out[0] = nf + sum_drho;
        out[1] = g_axis != 0.0 ? (1.0 / 6.0) * (sum_u / (double)n) / g_axis : 0.0;
        out[2] = nf;
        out[3] = acc[3];
    }
}

// Copy probe: one 16-byte vector per thread (the grid covers the array; the
// stride loop only runs for arrays beyond 2^30 vectors).
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
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
// Wall list (set-up, once per context): per (y, z) row, one entry for every
// fluid node with at least one solid lattice neighbour x + c_k (periodic), in
// increasing x.  The step kernel evaluates halfway bounce-back (Eq. 11) only
// at these nodes.  Entry bits: 0-9 x, 10-11 y mod G (the row's place in its
// lane-group block), 12.. one bit per direction k = 1..q-1, set when x + c_k
// is solid.  uint32 entries for D3Q15/19, uint64 for D3Q27.  One thread per
// row walks the row's 32-node words using the extended mask (bit e <-> node
// e - 1, periodic) of the neighbour rows.
// ---------------------------------------------------------------------------
template <int Q>
struct WallRow {
    uint32_t nb[Q];  // nb[k]: bit j set when node 32 w + j + c_k is solid
    uint32_t wall;   // fluid nodes of the word with a solid neighbour
};

template <int Q>
__device__ __forceinline__ void wall_word(const uint32_t* __restrict__ xm, int nx, int ny, int nz,
                                          int xwords, int y, int z, int w, WallRow<Q>& out) {
    using L = Lattice<Q>;
    auto window = [&](int yy, int zz) -> uint64_t {
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        const uint32_t* row = xm + ((int64_t)zz * ny + yy) * xwords;
        // node 32 w + j - 1 sits at bit j of this window
        return (uint64_t)row[w] | ((uint64_t)row[w + 1] << 32);
    };
    uint32_t any = 0;
    out.nb[0] = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        const Dir c = L::c[k];
        out.nb[k] = (uint32_t)(window(y + c.y, z + c.z) >> (1 + c.x));
        any |= out.nb[k];
    }
    const uint32_t own = (uint32_t)(window(y, z) >> 1);
    const int left = nx - 32 * w;
    const uint32_t valid = left >= 32 ? 0xffffffffu : ((1u << left) - 1u);
    out.wall = any & ~own & valid;
}

template <int Q>
__global__ void k_wall_count(const uint32_t* __restrict__ xm, int nx, int ny, int nz, int xwords,
                             uint32_t* __restrict__ count) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)ny * nz) return;
    const int y = (int)(r % ny), z = (int)(r / ny);
    uint32_t n = 0;
    for (int w = 0; w < (nx + 31) / 32; ++w) {
        WallRow<Q> wr;
        wall_word<Q>(xm, nx, ny, nz, xwords, y, z, w, wr);
        n += __builtin_popcount(wr.wall);
    }
    count[r] = n;
}

template <int Q, typename E>
__global__ void k_wall_fill(const uint32_t* __restrict__ xm, int nx, int ny, int nz, int xwords,
                            int G, const uint32_t* __restrict__ off, E* __restrict__ list) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)ny * nz) return;
    const int y = (int)(r % ny), z = (int)(r / ny);
    uint32_t at = off[r];
    for (int w = 0; w < (nx + 31) / 32; ++w) {
        WallRow<Q> wr;
        wall_word<Q>(xm, nx, ny, nz, xwords, y, z, w, wr);
        uint32_t b = wr.wall;
        while (b) {
            const int j = __builtin_ctz(b);
            b &= b - 1;
            E links = 0;
            for (int k = 1; k < Q; ++k) links |= (E)((wr.nb[k] >> j) & 1u) << (k - 1);
            list[at++] = (E)(32 * w + j) | ((E)(y % G) << 10) | (links << 12);
        }
    }
}

}  // namespace tau1
