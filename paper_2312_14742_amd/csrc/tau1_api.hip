// tau1_api.hip -- host side of the C ABI declared in include/tau1.h:
// descriptor validation, workspace planning, geometry encode and state
// upload, step launches and HIP graphs, readback and FP64 reductions,
// autotuning of the z-march tile shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tau1.h"
#include "tau1_device.hpp"
#include "tau1_kernels.hpp"
#include "tau1_zmarch.hpp"
#include "tau1_service.hpp"

using namespace tau1;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kStageNodes = int64_t(1) << 21;   // upload/readback chunk
constexpr int kMaxSamples = 1 << 16;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct SampleHost {
    SampleDev dev;
    int64_t n_fluid;
    std::vector<uint32_t> ctab;  // packed layout: chunk table (4 words per entry)
    int64_t nch = 0;             // packed layout: stored chunks
    bool ck = false;             // holds the chunk list and neighbour records
    std::vector<uint8_t> rowfluid;  // z-march samples: 1 if row y + ny z holds a fluid node
};

// Byte layout of the workspace for one descriptor.
struct Plan {
    size_t samples_off = 0;   // SampleDev[nsamples]
    size_t partial_off = 0;   // reduction partials + result + counters
    size_t tiles_off = 0;     // z-march work list
    size_t stage_off = 0;     // upload / readback staging
    size_t stage_bytes = 0;
    size_t total = 0;
    int64_t ntiles = 0;
    int64_t total_blocks = 0;
    bool packed = false;       // some sample uses the packed layout
    bool pack_refused = false; // packed layout requested but no sample qualifies
    std::vector<SampleHost> s;
};

// FP16 storage: stored = value * 2^s with s = 16 unless the descriptor sets
// it.  Half's largest finite value is 65504, so a state value must stay below
// 65504 * 2^-s; an initial field is accepted up to half of that, leaving the
// flow room to grow.
constexpr int kF16DefaultLog2Scale = 16;
int f16_log2_scale(int requested) { return requested ? requested : kF16DefaultLog2Scale; }
double f16_limit(int log2_scale) { return 0.5 * 65504.0 * std::ldexp(1.0, -log2_scale); }

bool valid_lattice(int q) { return q == 9 || q == 15 || q == 19 || q == 27; }
bool valid_precision(int p) { return p >= kF64 && p <= kBF16; }

tau1_status validate(const tau1_desc* d) {
    if (!d) return TAU1_E_INVALID;
    if (!valid_lattice(d->lattice) || !valid_precision(d->precision)) return TAU1_E_INVALID;
    if (d->n_samples < 1 || d->n_samples > kMaxSamples || !d->samples) return TAU1_E_INVALID;
    if (d->graph_chunk < 0 || (d->graph_chunk % 2) != 0) return TAU1_E_INVALID;
    if (d->kernel < -1 || d->kernel > 1) return TAU1_E_INVALID;
    if (d->tile < -1 || d->tile >= kNumTiles) return TAU1_E_INVALID;
    if (d->layout < -1 || d->layout > 1) return TAU1_E_INVALID;
    if (d->x_boundary < 0 || d->x_boundary > 1) return TAU1_E_INVALID;
    if (d->batch_graph < 0 || d->batch_graph > 3) return TAU1_E_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->wall_u[a])) return TAU1_E_INVALID;
    if (d->x_boundary == 1 &&
        !(std::isfinite(d->rho_in) && std::isfinite(d->rho_out) && d->rho_in > 0 &&
          d->rho_out > 0))
        return TAU1_E_INVALID;
    if (d->lattice == 9 && d->g[2] != 0.0) return TAU1_E_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->g[a])) return TAU1_E_INVALID;
    if (d->f16_log2_scale_rho < 0 || d->f16_log2_scale_rho > 40 ||
        d->f16_log2_scale_u < 0 || d->f16_log2_scale_u > 40)
        return TAU1_E_INVALID;
    for (int i = 0; i < d->n_samples; ++i) {
        const tau1_sample& s = d->samples[i];
        if (s.nx < 1 || s.ny < 1 || s.nz < 1 || !s.solid) return TAU1_E_INVALID;
        if (s.nx > (1 << 20) || s.ny > (1 << 20) || s.nz > (1 << 20)) return TAU1_E_INVALID;
        if (s.nx * s.ny > (int64_t(1) << 31)) return TAU1_E_INVALID;
        if (s.nx * s.ny * s.nz > (int64_t(1) << 36)) return TAU1_E_INVALID;
        if (d->lattice == 9 && s.nz != 1) return TAU1_E_INVALID;
        if (d->x_boundary == 1 && s.nx < 3) return TAU1_E_INVALID;
    }
    return TAU1_OK;
}

// Valid requests this build does not serve: the D2Q9 validation lattice has
// one kernel, in FP64 and FP32; its boundaries exist only there.
tau1_status unsupported(const tau1_desc* d) {
    if (d->lattice == 9 && (d->precision > kF32 || d->kernel != -1)) return TAU1_E_UNSUPPORTED;
    if (d->lattice != 9 && (d->x_boundary != 0 || d->wall_u[0] != 0.0 || d->wall_u[1] != 0.0 ||
                            d->wall_u[2] != 0.0))
        return TAU1_E_UNSUPPORTED;
    return TAU1_OK;
}

// Packed layout of one sample: its rows are cut into lane chunks of k nodes,
// `groups` groups of 64 chunks per row.  Returns the number of chunks holding
// a fluid node; with `tab` it also writes the chunk table (per row and group:
// fluid bitmap lo, hi, packed index of the group's first fluid chunk, 0).
int64_t chunk_table(const tau1_sample& in, int k, int groups, uint32_t* tab) {
    const int64_t rows = in.ny * in.nz;
    int64_t rank = 0;
    for (int64_t r = 0; r < rows; ++r) {
        const uint8_t* row = in.solid + r * in.nx;
        for (int g = 0; g < groups; ++g) {
            uint64_t bits = 0;
            for (int l = 0; l < 64; ++l) {
                // lanes past the row's end (layouts with idle lanes) hold no chunk
                const int64_t x0 = (int64_t)(g * 64 + l) * k;
                if (x0 >= in.nx) break;
                const uint8_t* ch = row + x0;
                bool fluid = false;
                for (int j = 0; j < k; ++j) fluid |= ch[j] == 0;
                bits |= (uint64_t)fluid << l;
            }
            if (tab) {
                uint32_t* e = tab + (r * groups + g) * 4;
                e[0] = (uint32_t)bits;
                e[1] = (uint32_t)(bits >> 32);
                e[2] = (uint32_t)rank;
                e[3] = 0;
            }
            rank += __builtin_popcountll(bits);
        }
    }
    return rank;
}

// Chunk list of a packed sample, built on the device from its chunk table:
// one thread per (row, group) entry writes the entries of its stored chunks.
__global__ void k_chunk_list(const ct_u4* __restrict__ tab, uint32_t* __restrict__ list,
                             int groups, int64_t entries) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= entries) return;
    const ct_u4 e = tab[i];
    uint64_t bits = ((uint64_t)e.y << 32) | e.x;
    const uint32_t row = (uint32_t)(i / groups), g = (uint32_t)(i % groups);
    uint32_t rank = e.z;
    while (bits) {
        const int l = __builtin_ctzll(bits);
        bits &= bits - 1u;
        list[rank++] = (row << kChunkBits) | (g * 64u + (uint32_t)l);
    }
}

// Neighbour-row records of a packed sample's stored chunks (the chunk
// tile's addressing), from its chunk table and list: one thread per stored
// chunk, nine records each (rows y + dy, z + dz, record (dy + 1) * 3 + dz + 1),
// stored as nine arrays of nch records.
__global__ void k_chunk_nbr(const ct_u4* __restrict__ tab, const uint32_t* __restrict__ list,
                            ck_rec_t* __restrict__ rec, int ny, int nz, int groups, int nrow,
                            int64_t nch) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nch) return;
    const uint32_t e = list[p];
    const int row = (int)(e >> kChunkBits), ci = (int)(e & ((1u << kChunkBits) - 1u));
    const int y = row % ny, z = row / ny;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
            const int yy = (y + dy + ny) % ny, zz = (z + dz + nz) % nz;
            const ct_u4* tr = tab + ((int64_t)zz * ny + yy) * groups;
            auto bits_of = [&](int g) { return ((uint64_t)tr[g].y << 32) | tr[g].x; };
            auto stored = [&](int cj) { return (uint32_t)((bits_of(cj >> 6) >> (cj & 63)) & 1u); };
            auto rank = [&](int cj) {
                const uint64_t below = bits_of(cj >> 6) & ((uint64_t(1) << (cj & 63)) - 1u);
                return tr[cj >> 6].z + (uint32_t)__popcll(below);
            };
            ck_rec_t r;
            r.x = rank(ci) | (ci > 0 ? stored(ci - 1) << 29 : 0u) | (stored(ci) << 30) |
                  (ci + 1 < nrow ? stored(ci + 1) << 31 : 0u);
            r.y = 0u;
            if (ci == 0 && stored(nrow - 1)) r.y = rank(nrow - 1) | (1u << 31);
            if (ci == nrow - 1 && stored(0)) r.y = rank(0) | (1u << 31);
            rec[(int64_t)((dy + 1) * 3 + dz + 1) * nch + p] = r;
        }
}

// Workspace plan; `tables` also builds the packed layout's chunk tables
// (the size query only counts chunks).
Plan make_plan(const tau1_desc* d, bool tables) {
    Plan p;
    const int sz = storage_bytes(d->precision);
    size_t off = 0;
    p.samples_off = off;
    off = align_up(off + sizeof(SampleDev) * d->n_samples, kAlign);
    p.partial_off = off;
    off = align_up(off + sizeof(double) * (kReduceBlocks * 4 + 8) + 64, kAlign);
    int64_t blocks = 0, tiles = 0, maxn = 0;
    p.s.resize(d->n_samples);
    for (int i = 0; i < d->n_samples; ++i) {
        const tau1_sample& in = d->samples[i];
        SampleDev& sd = p.s[i].dev;
        std::memset(&sd, 0, sizeof sd);
        sd.nx = (int32_t)in.nx;
        sd.ny = (int32_t)in.ny;
        sd.nz = (int32_t)in.nz;
        sd.n = in.nx * in.ny * in.nz;
        sd.words = (int32_t)((in.nx + 31) / 32);
        sd.stride = (int64_t)(align_up((size_t)sd.n * sz, kAlign) / sz);
        sd.block0 = blocks;
        blocks += (sd.n + kGatherBlock - 1) / kGatherBlock;
        zmarch_tiling(sd);
        if (d->lattice == 9) sd.variant = -1;  // the D2Q9 kernel only
        maxn = std::max<int64_t>(maxn, sd.n);
    }
    // packed layout: by default for the z-march precisions (FP32 and the
    // 16-bit storage modes) unless a dense-layout tile is asked for;
    // one-row-per-wave lane layouts only, and only where the z-march kernel
    // runs
    const bool zm = zmarch_supported(d->lattice, d->precision, p.s.data(), d->n_samples);
    const bool auto_pack = d->precision != kF64 && (d->tile < 0 || tile_packed(d->tile));
    const bool pack = zm && (d->kernel == -1 || d->kernel == 1) &&
                      (d->layout == 1 || (d->layout < 0 && auto_pack));
    // All samples of one lane layout share a launch, so a layout is packed
    // only if each of its samples fits: the step kernel addresses the four
    // packed arrays of a buffer with 32-bit offsets from one base.
    std::vector<int64_t> pstride(d->n_samples, 0);
    bool layout_ok[kNumVariants];
    for (int v = 0; v < kNumVariants; ++v) layout_ok[v] = pack && kVariants[v].g == 1;
    for (int i = 0; pack && i < d->n_samples; ++i) {
        const SampleDev& sd = p.s[i].dev;
        if (!layout_ok[sd.variant]) continue;
        const int k = kVariants[sd.variant].k;
        const int64_t nch = chunk_table(d->samples[i], k, kVariants[sd.variant].c, nullptr);
        p.s[i].nch = nch;
        pstride[i] = (int64_t)(align_up((size_t)std::max<int64_t>(nch * k, 1) * sz, kAlign) / sz);
        if (4 * pstride[i] * sz + 65536 > (int64_t)kOob) layout_ok[sd.variant] = false;
    }
    for (int i = 0; pack && i < d->n_samples; ++i) {
        SampleDev& sd = p.s[i].dev;
        if (!layout_ok[sd.variant]) continue;
        const int k = kVariants[sd.variant].k;
        const int groups = kVariants[sd.variant].c;
        if (tables) {
            p.s[i].ctab.assign((size_t)sd.ny * sd.nz * groups * 4, 0u);
            chunk_table(d->samples[i], k, groups, p.s[i].ctab.data());
        }
        sd.pk = k;
        sd.nchunks = p.s[i].nch;
        sd.stride = pstride[i];
        p.packed = true;
    }
    for (auto& sh : p.s)
        if (!sh.dev.pk) sh.nch = 0;  // counted, but its lane layout stays dense
    // The chunk tile's list and neighbour records (76 B per stored chunk):
    // where the chunk tile is asked for, or where at most half of the
    // sample's chunks are stored (the media the chunk tile is for).
    for (auto& sh : p.s) {
        if (!sh.dev.pk) continue;
        const int64_t all = (int64_t)sh.dev.ny * sh.dev.nz * (sh.dev.nx / sh.dev.pk);
        sh.ck = (d->tile == kChunkTile || 2 * sh.nch <= all) && sh.nch <= (int64_t)kRecIndex;
    }
    p.pack_refused = d->layout == 1 && !p.packed;
    // work-list capacity: the longest z-march list (16-plane segments) or the
    // chunk tile's list (one item per 64 stored chunks), whichever is longer
    tiles = zmarch_max_items(p.s.data(), d->n_samples);
    {
        int64_t ck = 0;
        for (const auto& sh : p.s)
            if (sh.ck) ck += (sh.nch + 63) / 64;
        tiles = std::max(tiles, ck);
    }
    p.total_blocks = blocks;
    p.ntiles = tiles;
    p.tiles_off = off;
    off = align_up(off + sizeof(int32_t) * 4 * (size_t)std::max<int64_t>(tiles, 1), kAlign);
    for (int i = 0; i < d->n_samples; ++i) {
        SampleDev& sd = p.s[i].dev;
        sd.mask = (int64_t)off;
        off = align_up(off + sizeof(uint32_t) * (size_t)sd.words * sd.ny * sd.nz, kAlign);
        sd.xmask = (int64_t)off;
        off = align_up(off + sizeof(uint32_t) * ((size_t)sd.xwords * sd.ny * sd.nz + 2), kAlign);
        if (sd.variant >= 0) {
            // wall list: row offsets, then at most one entry per node
            sd.wall_off = (int64_t)off;
            off = align_up(off + sizeof(uint32_t) * ((size_t)sd.ny * sd.nz + 1), kAlign);
            sd.wall_list = (int64_t)off;
            off = align_up(off + (d->lattice == 27 ? 8 : 4) * (size_t)sd.n + 8, kAlign);
        }
        if (sd.pk) {
            sd.chunk_tab = (int64_t)off;
            off = align_up(off + 16 * (size_t)sd.ny * sd.nz * kVariants[sd.variant].c, kAlign);
            if (p.s[i].ck) {
                const size_t nch = (size_t)std::max<int64_t>(p.s[i].nch, 1);
                sd.chunk_list = (int64_t)off;
                off = align_up(off + 4 * nch, kAlign);
                sd.chunk_nbr = (int64_t)off;
                off = align_up(off + 9 * 8 * nch, kAlign);
            }
        }
        if (d->lattice == 9) {
            sd.types = (int64_t)off;
            off = align_up(off + (size_t)sd.n, kAlign);
        }
        for (int b = 0; b < 2; ++b) {
            sd.state[b] = (int64_t)off;
            off = align_up(off + (size_t)4 * sd.stride * sz, kAlign);
        }
    }
    const int64_t stage_nodes = std::min<int64_t>(maxn, kStageNodes);
    p.stage_off = off;
    // solid byte + drho + 3 u (FP64) on upload; 4 FP64 on readback
    p.stage_bytes = align_up((size_t)stage_nodes * 40 + kAlign, kAlign);
    off += p.stage_bytes;
    p.total = off;
    return p;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return fail_hip(ctx, _e); \
    } while (0)

}  // namespace

// Device scratch of tau1_permeability_noalloc: the reduction's block
// partials, kReduceBlocks x 4 doubles = 32 KiB.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the name stands
// for no device address: kernels get the address that hipGetSymbolAddress
// reports for the current device (scratch_on_device).
constexpr int kScratchDoubles = kReduceBlocks * 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up once per device (at
// the first tau1_create on it); nullptr if the lookup failed.
double* scratch_on_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
            g_scratch_ptr[dev] = static_cast<double*>(p);
        else
            (void)hipGetLastError();
    }
    return g_scratch_ptr[dev];
}

}  // namespace

struct tau1_ctx {
    int lattice = 19, precision = kF32, nsamples = 1;
    int graph_chunk = 100;
    int kernel = 0, tile = 0;
    hipStream_t stream = nullptr;
    uint8_t* base = nullptr;
    size_t ws_bytes = 0;
    Plan plan;
    StepArgs args[2];
    // z-march launches: one per lane layout present, each over its samples' items
    struct ZGroup {
        int variant;
        int tile;     // its tile (the autotuner picks one per lane layout)
        bool packed;  // its samples use the packed layout
        bool chunks;  // ... and hold the chunk tile's list and records
        int rows_mode = -1;  // >= 0: several one-row layouts in one launch
                             // (k_zmarch_rows in this mode); variant, tile are
                             // then those of the layout with the most work
        StepArgs args[2];
    };
    std::vector<ZGroup> zgroups;
    int parity = 0;
    int64_t steps_done = 0;
    int64_t n_nodes = 0, n_fluid = 0;
    tau1_status sticky = TAU1_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_kernel = -1, graph_tile = -1, graph_parity = -1;
    bool graph_chains = false;  // batch graphs: one chain per lane layout (else one chain)
    bool merge_rows = false;    // one launch for the one-row layouts of a batch
    double g[3] = {0, 0, 0};
    std::string cache;
    hipError_t last_hip = hipSuccess;
    double* scratch = nullptr;  // this context's device's copy of `scratch`
};

namespace {

tau1_status fail_hip(tau1_ctx* ctx, hipError_t e) {
    if (ctx) {
        ctx->sticky = TAU1_E_HIP;
        ctx->last_hip = e;
    }
    (void)hipGetLastError();
    return TAU1_E_HIP;
}

// --- kernel dispatch -------------------------------------------------------
template <int Q, int P>
void* gather_fn() { return reinterpret_cast<void*>(&k_gather<Q, P>); }

void* pick_gather(int q, int p) {
    switch (q * 10 + p) {
        case 150: return gather_fn<15, kF64>();
        case 151: return gather_fn<15, kF32>();
        case 152: return gather_fn<15, kF16>();
        case 153: return gather_fn<15, kBF16>();
        case 190: return gather_fn<19, kF64>();
        case 191: return gather_fn<19, kF32>();
        case 192: return gather_fn<19, kF16>();
        case 193: return gather_fn<19, kBF16>();
        case 270: return gather_fn<27, kF64>();
        case 271: return gather_fn<27, kF32>();
        case 272: return gather_fn<27, kF16>();
        case 273: return gather_fn<27, kBF16>();
    }
    return nullptr;
}

// Launch geometry of one step for the chosen kernel.
struct Launch {
    void* fn;
    dim3 grid, block;
    size_t shmem;
};

bool zmarch_eligible(const tau1_ctx* ctx) {
    return zmarch_supported(ctx->lattice, ctx->precision, ctx->plan.s.data(),
                            (int)ctx->plan.s.size());
}

void* pick_d2q9(int p) {
    switch (p) {
        case kF64: return reinterpret_cast<void*>(&k_d2q9<kF64>);
        case kF32: return reinterpret_cast<void*>(&k_d2q9<kF32>);
    }
    return nullptr;
}

// Load mode of group g's z-march kernel (a dense one-row layout in a packed
// context runs the dense shared-row schedule), or -1 for the chunk kernel.
int group_mode(const tau1_ctx::ZGroup& g) {
    if (g.tile == kChunkTile && g.chunks) return -1;
    const int zt = tile_zmarch(g.tile);
    return tile_mode(zt) == 3 && !g.packed ? 1 : tile_mode(zt);
}

// Launch geometry of one step kernel: z-march group g (kernel 1), the
// per-node gather over every sample (kernel 0) or the D2Q9 kernel (2).
Launch step_launch(const tau1_ctx* ctx, int kernel, int tile, int g) {
    Launch l{};
    if (kernel == 1) tile = ctx->zgroups[g].tile;
    if (kernel == 1 && tile == kChunkTile && ctx->zgroups[g].chunks) {
        const auto& grp = ctx->zgroups[g];
        l.fn = pick_chunks(ctx->lattice, ctx->precision, kVariants[grp.variant].k);
        l.block = dim3(kCkThreads);
        l.grid = dim3((unsigned)((grp.args[0].ntiles + kCkWaves - 1) / kCkWaves));
        l.shmem = 0;
    } else if (kernel == 1 && ctx->zgroups[g].rows_mode >= 0) {
        const auto& grp = ctx->zgroups[g];
        l.fn = pick_zmarch_rows(ctx->lattice, ctx->precision, grp.rows_mode);
        l.block = dim3(kZrThreads);
        l.grid = dim3((unsigned)zmarch_grid(grp.args[0].ntiles, tile));
        l.shmem = 0;
    } else if (kernel == 1) {
        const auto& grp = ctx->zgroups[g];
        tile = tile_zmarch(tile);
        l.fn = pick_zmarch(ctx->lattice, ctx->precision, grp.variant, group_mode(grp));
        l.block = dim3(zmarch_threads(tile));
        l.grid = dim3((unsigned)zmarch_grid(grp.args[0].ntiles, tile));
        l.shmem = 0;
    } else {
        l.fn = kernel == 2 ? pick_d2q9(ctx->precision) : pick_gather(ctx->lattice, ctx->precision);
        l.block = dim3(kGatherBlock);
        l.grid = dim3((unsigned)ctx->plan.total_blocks);
        l.shmem = 0;
    }
    return l;
}

int launch_groups(const tau1_ctx* ctx, int kernel) {
    return kernel == 1 ? (int)ctx->zgroups.size() : 1;
}

StepArgs* launch_args(tau1_ctx* ctx, int kernel, int g, int parity) {
    return kernel == 1 ? &ctx->zgroups[g].args[parity] : &ctx->args[parity];
}

// One time step reading buffer `parity`: every launch of the step in order.
tau1_status launch_one(tau1_ctx* ctx, int kernel, int tile, int parity) {
    for (int g = 0; g < launch_groups(ctx, kernel); ++g) {
        const Launch l = step_launch(ctx, kernel, tile, g);
        if (!l.fn) return TAU1_E_UNSUPPORTED;
        if (l.grid.x == 0) continue;
        void* params[] = {launch_args(ctx, kernel, g, parity)};
        HIP_TRY(hipLaunchKernel(l.fn, l.grid, l.block, params, l.shmem, ctx->stream));
    }
    return TAU1_OK;
}

// Whether some sample holds the chunk tile's list and records.
bool any_chunks(const tau1_ctx* ctx) {
    for (const auto& sh : ctx->plan.s)
        if (sh.dev.chunk_list) return true;
    return false;
}

// The launch of lane-layout group g alone (autotune trials).
tau1_status launch_group(tau1_ctx* ctx, int g, int parity) {
    const Launch l = step_launch(ctx, 1, ctx->zgroups[g].tile, g);
    if (!l.fn) return TAU1_E_UNSUPPORTED;
    if (l.grid.x == 0) return TAU1_OK;
    void* params[] = {launch_args(ctx, 1, g, parity)};
    HIP_TRY(hipLaunchKernel(l.fn, l.grid, l.block, params, l.shmem, ctx->stream));
    return TAU1_OK;
}

void destroy_graph(tau1_ctx* ctx) {
    if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_kernel = ctx->graph_tile = -1;
}

// Graph of graph_chunk time steps.  The parity alternates step by step and,
// graph_chunk being even, the graph maps the current buffer onto itself.
// A context with several launch groups (a batch of several z-march lane
// layouts) either runs them as one chain -- the launches of a step one after
// another, each with the whole GPU -- or as one chain per group, the chains
// side by side (the groups share no samples, so they are independent).
// Built without stream capture.
tau1_status build_graph(tau1_ctx* ctx) {
    destroy_graph(ctx);
    HIP_TRY(hipGraphCreate(&ctx->graph, 0));
    const int ng = launch_groups(ctx, ctx->kernel);
    std::vector<Launch> ls;
    for (int g = 0; g < ng; ++g) {
        ls.push_back(step_launch(ctx, ctx->kernel, ctx->tile, g));
        if (!ls.back().fn) return TAU1_E_UNSUPPORTED;
    }
    auto add = [&](int g, int s, hipGraphNode_t* prev) -> tau1_status {
        const Launch& l = ls[g];
        void* params[] = {launch_args(ctx, ctx->kernel, g, (ctx->parity + s) & 1)};
        hipKernelNodeParams kp{};
        kp.func = l.fn;
        kp.gridDim = l.grid;
        kp.blockDim = l.block;
        kp.sharedMemBytes = (unsigned)l.shmem;
        kp.kernelParams = params;
        kp.extra = nullptr;
        hipGraphNode_t node;
        HIP_TRY(hipGraphAddKernelNode(&node, ctx->graph, *prev ? prev : nullptr, *prev ? 1 : 0,
                                      &kp));
        *prev = node;
        return TAU1_OK;
    };
    if (ctx->graph_chains || ng == 1) {
        for (int g = 0; g < ng; ++g) {
            if (ls[g].grid.x == 0) continue;
            hipGraphNode_t prev = nullptr;
            for (int s = 0; s < ctx->graph_chunk; ++s) {
                const tau1_status st = add(g, s, &prev);
                if (st != TAU1_OK) return st;
            }
        }
    } else {
        // groups in the order of launch_one (largest work first)
        hipGraphNode_t prev = nullptr;
        for (int s = 0; s < ctx->graph_chunk; ++s)
            for (int g = 0; g < ng; ++g) {
                if (ls[g].grid.x == 0) continue;
                const tau1_status st = add(g, s, &prev);
                if (st != TAU1_OK) return st;
            }
    }
    HIP_TRY(hipGraphInstantiate(&ctx->exec, ctx->graph, nullptr, nullptr, 0));
    ctx->graph_kernel = ctx->kernel;
    ctx->graph_tile = ctx->tile;
    ctx->graph_parity = ctx->parity;
    return TAU1_OK;
}

// Wall list of one sample (z-march samples only): count per row on the GPU,
// exclusive scan of the row counts on the host, fill on the GPU.
template <int Q>
tau1_status build_wall_list_q(tau1_ctx* ctx, const SampleDev& sd) {
    const int64_t rows = (int64_t)sd.ny * sd.nz;
    uint32_t* off = reinterpret_cast<uint32_t*>(ctx->base + sd.wall_off);
    const uint32_t* xm = reinterpret_cast<const uint32_t*>(ctx->base + sd.xmask);
    using E = typename WallEntry<Q>::type;
    E* list = reinterpret_cast<E*>(ctx->base + sd.wall_list);
    const unsigned grid = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(k_wall_count<Q>, dim3(grid), dim3(256), 0, ctx->stream, xm, sd.nx, sd.ny,
                       sd.nz, sd.xwords, off);
    HIP_TRY(hipGetLastError());
    std::vector<uint32_t> h;
    try {
        h.resize((size_t)rows + 1);
    } catch (const std::bad_alloc&) {
        return TAU1_E_NOMEM;
    }
    HIP_TRY(hipMemcpyAsync(h.data(), off, sizeof(uint32_t) * rows, hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    uint64_t acc = 0;
    for (int64_t r = 0; r < rows; ++r) {
        const uint32_t c = h[r];
        h[r] = (uint32_t)acc;
        acc += c;
    }
    if (acc > (uint64_t)sd.n) return TAU1_E_INVALID;  // cannot happen: one entry per node at most
    h[rows] = (uint32_t)acc;
    HIP_TRY(hipMemcpyAsync(off, h.data(), sizeof(uint32_t) * (rows + 1), hipMemcpyHostToDevice,
                           ctx->stream));
    hipLaunchKernelGGL((k_wall_fill<Q, E>), dim3(grid), dim3(256), 0, ctx->stream, xm, sd.nx,
                       sd.ny, sd.nz, sd.xwords, kVariants[sd.variant].g, off, list);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TAU1_OK;
}

tau1_status build_wall_list(tau1_ctx* ctx, const SampleDev& sd) {
    switch (ctx->lattice) {
        case 15: return build_wall_list_q<15>(ctx, sd);
        case 19: return build_wall_list_q<19>(ctx, sd);
        case 27: return build_wall_list_q<27>(ctx, sd);
    }
    return TAU1_E_INVALID;
}

template <int P>
tau1_status upload_sample_t(tau1_ctx* ctx, int s, const tau1_sample& in) {
    const SampleDev& sd = ctx->plan.s[s].dev;
    uint8_t* stage = ctx->base + ctx->plan.stage_off;
    const int64_t n = sd.n;
    const int64_t chunk = std::min<int64_t>(n, kStageNodes);
    // geometry: whole rows per chunk
    const int64_t rows = (int64_t)sd.ny * sd.nz;
    const int64_t rows_per = std::max<int64_t>(1, chunk / sd.nx);
    uint32_t* mask = reinterpret_cast<uint32_t*>(ctx->base + sd.mask);
    for (int64_t r0 = 0; r0 < rows; r0 += rows_per) {
        const int64_t nr = std::min(rows_per, rows - r0);
        HIP_TRY(hipMemcpyAsync(stage, in.solid + r0 * sd.nx, (size_t)(nr * sd.nx),
                               hipMemcpyHostToDevice, ctx->stream));
        const int64_t nt = nr * sd.words;
        hipLaunchKernelGGL(k_pack_mask, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                           ctx->stream, stage, mask, sd.nx, sd.words, r0, nr);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    {
        const int64_t nt = rows * sd.xwords;
        uint32_t* xm = reinterpret_cast<uint32_t*>(ctx->base + sd.xmask);
        hipLaunchKernelGGL(k_build_xmask, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                           ctx->stream, mask, xm, sd.nx, sd.words, sd.xwords, rows);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemsetAsync(xm + nt, 0, 2 * sizeof(uint32_t), ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    if (sd.variant >= 0) {
        const tau1_status st = build_wall_list(ctx, sd);
        if (st != TAU1_OK) return st;
    }
    if (sd.types) {
        HIP_TRY(hipMemcpyAsync(ctx->base + sd.types, in.solid, (size_t)n, hipMemcpyHostToDevice,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    if (sd.pk) {
        const auto& tab = ctx->plan.s[s].ctab;
        HIP_TRY(hipMemcpyAsync(ctx->base + sd.chunk_tab, tab.data(), sizeof(uint32_t) * tab.size(),
                               hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    if (sd.chunk_list) {
        // chunk list (the chunk tile's work) and neighbour records, from the
        // table on the device
        const int groups = kVariants[sd.variant].c;
        const int64_t entries = (int64_t)sd.ny * sd.nz * groups;
        const ct_u4* tab = reinterpret_cast<const ct_u4*>(ctx->base + sd.chunk_tab);
        uint32_t* list = reinterpret_cast<uint32_t*>(ctx->base + sd.chunk_list);
        hipLaunchKernelGGL(k_chunk_list, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0,
                           ctx->stream, tab, list, groups, entries);
        HIP_TRY(hipGetLastError());
        const int64_t nch = ctx->plan.s[s].nch;
        if (nch > 0) {
            hipLaunchKernelGGL(k_chunk_nbr, dim3((unsigned)((nch + 255) / 256)), dim3(256), 0,
                               ctx->stream, tab, list,
                               reinterpret_cast<ck_rec_t*>(ctx->base + sd.chunk_nbr), sd.ny, sd.nz,
                               groups, sd.nx / sd.pk, nch);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    // state (the packed layout's upload kernel skips nodes of all-solid chunks)
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
        const int64_t len = std::min(chunk, n - i0);
        uint8_t* st_solid = stage;
        double* st_d = reinterpret_cast<double*>(stage + align_up((size_t)len, kAlign));
        double* st_u = st_d + len;
        HIP_TRY(hipMemcpyAsync(st_solid, in.solid + i0, (size_t)len, hipMemcpyHostToDevice,
                               ctx->stream));
        if (in.drho0)
            HIP_TRY(hipMemcpyAsync(st_d, in.drho0 + i0, sizeof(double) * len,
                                   hipMemcpyHostToDevice, ctx->stream));
        if (in.u0) {
            // D2Q9: two velocity components; the third is held at zero
            const int ncomp = ctx->lattice == 9 ? 2 : 3;
            for (int a = 0; a < ncomp; ++a)
                HIP_TRY(hipMemcpyAsync(st_u + a * len, in.u0 + (int64_t)a * n + i0,
                                       sizeof(double) * len, hipMemcpyHostToDevice,
                                       ctx->stream));
            if (ncomp == 2)
                HIP_TRY(hipMemsetAsync(st_u + 2 * len, 0, sizeof(double) * len, ctx->stream));
        }
        hipLaunchKernelGGL(k_upload<P>, dim3((unsigned)((len + 255) / 256)), dim3(256), 0,
                           ctx->stream, ctx->args[0], s, st_solid, in.drho0 ? st_d : nullptr,
                           in.u0 ? st_u : nullptr, i0, len);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    return TAU1_OK;
}

tau1_status upload_sample(tau1_ctx* ctx, int s, const tau1_sample& in) {
    switch (ctx->precision) {
        case kF64: return upload_sample_t<kF64>(ctx, s, in);
        case kF32: return upload_sample_t<kF32>(ctx, s, in);
        case kF16: return upload_sample_t<kF16>(ctx, s, in);
        case kBF16: return upload_sample_t<kBF16>(ctx, s, in);
    }
    return TAU1_E_INVALID;
}

template <int P>
tau1_status export_sample_t(tau1_ctx* ctx, int s, double* drho, double* u, int* nbad,
                            bool phys_rho) {
    const SampleDev& sd = ctx->plan.s[s].dev;
    uint8_t* stage = ctx->base + ctx->plan.stage_off;
    int* bad = reinterpret_cast<int*>(ctx->base + ctx->plan.partial_off +
                                      sizeof(double) * (kReduceBlocks * 4 + 4));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    const int64_t n = sd.n;
    const int64_t chunk = std::min<int64_t>(n, kStageNodes);
    double* out = reinterpret_cast<double*>(stage);
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
        const int64_t len = std::min(chunk, n - i0);
        hipLaunchKernelGGL(k_export<P>, dim3((unsigned)((len + 255) / 256)), dim3(256), 0,
                           ctx->stream, ctx->args[ctx->parity], s, out, i0, len, bad,
                           phys_rho ? 1 : 0);
        HIP_TRY(hipGetLastError());
        if (drho)
            HIP_TRY(hipMemcpyAsync(drho + i0, out, sizeof(double) * len, hipMemcpyDeviceToHost,
                                   ctx->stream));
        if (u)
            for (int a = 0; a < 3; ++a)
                HIP_TRY(hipMemcpyAsync(u + (int64_t)a * n + i0, out + (1 + a) * len,
                                       sizeof(double) * len, hipMemcpyDeviceToHost,
                                       ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    HIP_TRY(hipMemcpyAsync(nbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TAU1_OK;
}

// Enqueues the two reduction kernels of one sample: block partials into
// `partial` (kReduceBlocks x 4 doubles, every entry written), then the four
// results into `res`.
template <int P>
tau1_status reduce_launch_t(tau1_ctx* ctx, int s, int axis, double* partial, double* res) {
    const SampleDev& sd = ctx->plan.s[s].dev;
    hipLaunchKernelGGL(k_reduce_partial<P>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                       ctx->stream, ctx->args[ctx->parity], s, axis, partial);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, ctx->stream, partial,
                       sd.n, ctx->g[axis], res);
    HIP_TRY(hipGetLastError());
    return TAU1_OK;
}

tau1_status reduce_launch(tau1_ctx* ctx, int s, int axis, double* partial, double* res) {
    switch (ctx->precision) {
        case kF64: return reduce_launch_t<kF64>(ctx, s, axis, partial, res);
        case kF32: return reduce_launch_t<kF32>(ctx, s, axis, partial, res);
        case kF16: return reduce_launch_t<kF16>(ctx, s, axis, partial, res);
        case kBF16: return reduce_launch_t<kBF16>(ctx, s, axis, partial, res);
    }
    return TAU1_E_INVALID;
}

// tau1_permeability's reduction: partials and results in the workspace.
tau1_status reduce_ws(tau1_ctx* ctx, int s, int axis, double out[4]) {
    double* partial = reinterpret_cast<double*>(ctx->base + ctx->plan.partial_off);
    double* res = partial + kReduceBlocks * 4;
    const tau1_status st = reduce_launch(ctx, s, axis, partial, res);
    if (st != TAU1_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, res, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TAU1_OK;
}

// Selects the tile of every lane layout (`tile`, or per_variant[v] where
// that is given and not negative), rebuilds and uploads the work lists;
// cached graphs are rebuilt on the next step.  The context's tile is that of
// the layout with the most fluid nodes.  With `merge`, the one-row, one-chunk
// layouts whose tiles run the shared-row schedule of one mode (that of the
// layout with the most work among them) share one launch, k_zmarch_rows,
// over their lists laid end to end; the other layouts launch alone.
tau1_status set_tile(tau1_ctx* ctx, int tile, const int* per_variant = nullptr,
                     bool merge = false) {
    // lane layouts present, the one with the most fluid nodes first (the
    // order of the launches of a step when they run one after another)
    std::vector<int> layouts;
    std::vector<int64_t> work(kNumVariants, 0);
    for (const auto& sh : ctx->plan.s) {
        if (sh.dev.variant < 0) continue;
        if (std::find(layouts.begin(), layouts.end(), sh.dev.variant) == layouts.end())
            layouts.push_back(sh.dev.variant);
        work[sh.dev.variant] += sh.n_fluid;
    }
    std::stable_sort(layouts.begin(), layouts.end(),
                     [&](int a, int b) { return work[a] > work[b]; });
    std::vector<tau1_ctx::ZGroup> groups;
    std::vector<std::vector<int32_t>> parts;
    for (int v : layouts) {
        tau1_ctx::ZGroup g;
        g.variant = v;
        g.tile = per_variant && per_variant[v] >= 0 ? per_variant[v] : tile;
        g.packed = false;
        g.chunks = true;
        for (const auto& sh : ctx->plan.s)
            if (sh.dev.variant == v) {
                if (sh.dev.pk) g.packed = true;
                if (!sh.dev.chunk_list) g.chunks = false;
            }
        g.chunks = g.chunks && g.packed;
        std::vector<int32_t> part;
        if (g.tile == kChunkTile && g.chunks) {
            // the chunk kernel: one item per 64 stored chunks of a sample
            for (int i = 0; i < ctx->nsamples; ++i) {
                const auto& sh = ctx->plan.s[i];
                if (sh.dev.variant != v) continue;
                for (int64_t c0 = 0; c0 < sh.nch; c0 += 64) {
                    part.push_back(i);
                    part.push_back((int32_t)c0);
                    part.push_back((int32_t)std::min<int64_t>(64, sh.nch - c0));
                    part.push_back(0);
                }
            }
        } else {
            const int zt = tile_zmarch(g.tile);
            part = zmarch_worklist(ctx->plan.s.data(), ctx->nsamples, tile_lz(zt), v,
                                   zr_share(kVariants[v].g, tile_mode(zt)));
        }
        groups.push_back(g);
        parts.push_back(std::move(part));
    }
    // the groups of the one launch, if any (at least two layouts)
    std::vector<bool> merged(groups.size(), false);
    int rows_mode = -1, nmerged = 0;
    if (merge) {
        for (size_t i = 0; i < groups.size(); ++i) {
            const int m = group_mode(groups[i]);
            if (!zr_rows_layout(kVariants[groups[i].variant]) || (m != 1 && m != 3)) continue;
            if (rows_mode < 0) rows_mode = m;
            if (m != rows_mode) continue;
            // whole blocks of kZrWaves row items, so a block never straddles two layouts
            if (parts[i].size() % (4 * kZrWaves) != 0) return TAU1_E_INVALID;
            merged[i] = true;
            ++nmerged;
        }
        if (nmerged < 2) merged.assign(groups.size(), false);
    }
    std::vector<int32_t> tl;
    std::vector<tau1_ctx::ZGroup> launches;
    auto add_launch = [&](tau1_ctx::ZGroup g, int64_t item0) {
        for (int p = 0; p < 2; ++p) {
            g.args[p] = ctx->args[p];
            g.args[p].tiles = reinterpret_cast<const int32_t*>(ctx->base + ctx->plan.tiles_off) +
                              4 * item0;
            g.args[p].ntiles = (int32_t)((int64_t)tl.size() / 4 - item0);
        }
        launches.push_back(g);
    };
    if (nmerged >= 2) {
        tau1_ctx::ZGroup g;
        bool lead = true;
        for (size_t i = 0; i < groups.size(); ++i) {
            if (!merged[i]) continue;
            if (lead) g = groups[i];
            lead = false;
            tl.insert(tl.end(), parts[i].begin(), parts[i].end());
        }
        g.rows_mode = rows_mode;
        add_launch(g, 0);
    }
    for (size_t i = 0; i < groups.size(); ++i) {
        if (merged[i]) continue;
        const int64_t item0 = (int64_t)tl.size() / 4;
        tl.insert(tl.end(), parts[i].begin(), parts[i].end());
        add_launch(groups[i], item0);
    }
    const int64_t items = (int64_t)tl.size() / 4;
    if (items > ctx->plan.ntiles) return TAU1_E_INVALID;
    if (!tl.empty()) {
        HIP_TRY(hipMemcpyAsync(ctx->base + ctx->plan.tiles_off, tl.data(),
                               sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    destroy_graph(ctx);
    ctx->zgroups.swap(launches);
    ctx->args[0].ntiles = ctx->args[1].ntiles = (int32_t)items;
    ctx->tile = ctx->zgroups.empty() ? tile : ctx->zgroups[0].tile;
    return TAU1_OK;
}

tau1_status check_usable(const tau1_ctx* ctx) {
    if (!ctx) return TAU1_E_INVALID;
    if (ctx->sticky != TAU1_OK) return ctx->sticky;
    return TAU1_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* tau1_strerror(tau1_status s) {
    switch (s) {
        case TAU1_OK: return "ok";
        case TAU1_E_INVALID: return "invalid argument";
        case TAU1_E_NOMEM: return "host allocation failed";
        case TAU1_E_HIP: return "HIP runtime or kernel error";
        case TAU1_E_UNSUPPORTED: return "unsupported configuration";
        case TAU1_E_NONFINITE: return "non-finite value in state or reduction";
        case TAU1_E_WORKSPACE: return "workspace missing, too small or misaligned";
    }
    return "unknown status";
}

tau1_status tau1_workspace_size(const tau1_desc* desc, size_t* bytes) {
    if (!bytes) return TAU1_E_INVALID;
    tau1_status v = validate(desc);
    if (v == TAU1_OK) v = unsupported(desc);
    if (v != TAU1_OK) return v;
    try {
        const Plan p = make_plan(desc, false);
        if (p.pack_refused) return TAU1_E_UNSUPPORTED;
        *bytes = p.total;
    } catch (const std::bad_alloc&) {
        return TAU1_E_NOMEM;
    }
    return TAU1_OK;
}

tau1_status tau1_create(const tau1_desc* desc, tau1_ctx** out) {
    if (!out) return TAU1_E_INVALID;
    *out = nullptr;
    tau1_status v = validate(desc);
    if (v == TAU1_OK) v = unsupported(desc);
    if (v != TAU1_OK) return v;
    // non-finite initial fields, and for FP16 storage fields beyond its range
    // at the chosen scales, are rejected before any GPU work
    const bool f16 = desc->precision == kF16;
    const double lim_r = f16_limit(f16_log2_scale(desc->f16_log2_scale_rho));
    const double lim_u = f16_limit(f16_log2_scale(desc->f16_log2_scale_u));
    for (int i = 0; i < desc->n_samples; ++i) {
        const tau1_sample& s = desc->samples[i];
        const int64_t n = s.nx * s.ny * s.nz;
        if (s.drho0)
            for (int64_t j = 0; j < n; ++j) {
                if (!std::isfinite(s.drho0[j]) || s.drho0[j] <= -1.0) return TAU1_E_INVALID;
                if (f16 && !s.solid[j] && std::fabs(s.drho0[j]) >= lim_r) return TAU1_E_INVALID;
            }
        if (s.u0)
            for (int64_t j = 0; j < 3 * n; ++j)
                if (!std::isfinite(s.u0[j])) return TAU1_E_INVALID;
        if (f16)
            for (int a = 0; a < 3; ++a) {
                const double gh = 0.5 * desc->g[a];
                if (std::fabs(gh) >= lim_u) return TAU1_E_INVALID;
                if (!s.u0) continue;
                for (int64_t j = 0; j < n; ++j)
                    if (!s.solid[j] && std::fabs(s.u0[(int64_t)a * n + j] + gh) >= lim_u)
                        return TAU1_E_INVALID;
            }
    }
    if (!desc->workspace) return TAU1_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(desc->workspace) % kAlign != 0) return TAU1_E_WORKSPACE;
    tau1_ctx* ctx = new (std::nothrow) tau1_ctx();
    if (!ctx) return TAU1_E_NOMEM;
    try {
        ctx->plan = make_plan(desc, true);
    } catch (const std::bad_alloc&) {
        delete ctx;
        return TAU1_E_NOMEM;
    }
    if (ctx->plan.pack_refused) {
        delete ctx;
        return TAU1_E_UNSUPPORTED;
    }
    // an explicit tile must belong to the context's layout
    if (desc->tile >= 0 && desc->kernel != 0 &&
        zmarch_supported(desc->lattice, desc->precision, ctx->plan.s.data(), desc->n_samples) &&
        !zmarch_tile_ok(desc->precision, ctx->plan.packed, desc->tile)) {
        delete ctx;
        return TAU1_E_INVALID;
    }
    if (desc->workspace_bytes < ctx->plan.total) {
        delete ctx;
        return TAU1_E_WORKSPACE;
    }
    // the allocation-free reduction's scratch on this device (once per device)
    ctx->scratch = scratch_on_device();
    ctx->lattice = desc->lattice;
    ctx->precision = desc->precision;
    ctx->nsamples = desc->n_samples;
    ctx->graph_chunk = desc->graph_chunk ? desc->graph_chunk : 100;
    ctx->stream = reinterpret_cast<hipStream_t>(desc->hip_stream);
    ctx->base = reinterpret_cast<uint8_t*>(desc->workspace);
    ctx->ws_bytes = desc->workspace_bytes;
    ctx->cache = desc->tune_cache ? desc->tune_cache : "";
    ctx->graph_chains = desc->batch_graph != 1;
    ctx->merge_rows = desc->batch_graph == 3;
    for (int a = 0; a < 3; ++a) ctx->g[a] = desc->g[a];

    const int lsr = f16_log2_scale(desc->f16_log2_scale_rho);
    const int lsu = f16_log2_scale(desc->f16_log2_scale_u);
    for (int p = 0; p < 2; ++p) {
        StepArgs& a = ctx->args[p];
        std::memset(&a, 0, sizeof a);
        a.base = ctx->base;
        a.samples = reinterpret_cast<const SampleDev*>(ctx->base + ctx->plan.samples_off);
        a.tiles = reinterpret_cast<const int32_t*>(ctx->base + ctx->plan.tiles_off);
        a.nsamples = ctx->nsamples;
        a.ntiles = (int32_t)ctx->plan.ntiles;
        a.parity = p;
        for (int d = 0; d < 3; ++d) {
            a.gh[d] = 0.5 * desc->g[d];
            a.ghf[d] = (float)(0.5 * desc->g[d]);
        }
        a.scale_rho = std::ldexp(1.0f, lsr);
        a.inv_scale_rho = std::ldexp(1.0f, -lsr);
        a.scale_u = std::ldexp(1.0f, lsu);
        a.inv_scale_u = std::ldexp(1.0f, -lsu);
        a.xbc = desc->x_boundary;
        a.din = desc->x_boundary ? desc->rho_in - 1.0 : 0.0;
        a.dout = desc->x_boundary ? desc->rho_out - 1.0 : 0.0;
        a.uw[0] = desc->wall_u[0];
        a.uw[1] = desc->wall_u[1];
    }
    // fluid counts, and for z-march samples the rows holding a fluid node
    // (host marshalling of the geometry)
    for (int i = 0; i < ctx->nsamples; ++i) {
        const tau1_sample& s = desc->samples[i];
        const int64_t rows = s.ny * s.nz;
        SampleHost& sh = ctx->plan.s[i];
        const bool rowflags = sh.dev.variant >= 0;
        try {
            if (rowflags) sh.rowfluid.assign((size_t)rows, 0);
        } catch (const std::bad_alloc&) {
            delete ctx;
            return TAU1_E_NOMEM;
        }
        int64_t nf = 0;
        for (int64_t r = 0; r < rows; ++r) {
            const uint8_t* row = s.solid + r * s.nx;
            int64_t c = 0;
            for (int64_t x = 0; x < s.nx; ++x) c += row[x] ? 0 : 1;
            nf += c;
            if (rowflags) sh.rowfluid[(size_t)r] = c != 0;
        }
        sh.n_fluid = nf;
        ctx->n_fluid += nf;
        ctx->n_nodes += rows * s.nx;
    }
    // descriptors
    std::vector<SampleDev> sdev(ctx->nsamples);
    for (int i = 0; i < ctx->nsamples; ++i) sdev[i] = ctx->plan.s[i].dev;
    tau1_status st = TAU1_OK;
    {
        hipError_t e = hipMemcpyAsync(ctx->base + ctx->plan.samples_off, sdev.data(),
                                      sizeof(SampleDev) * sdev.size(), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = fail_hip(ctx, e);
    }
    for (int i = 0; st == TAU1_OK && i < ctx->nsamples; ++i)
        st = upload_sample(ctx, i, desc->samples[i]);
    if (st != TAU1_OK) {
        delete ctx;
        return st;
    }
    // kernel choice: explicit, else tuned cache, else the default
    const bool zm = zmarch_eligible(ctx);
    if (desc->kernel == 1 && !zm) {
        delete ctx;
        return TAU1_E_UNSUPPORTED;
    }
    ctx->kernel = ctx->lattice == 9 ? 2 : desc->kernel >= 0 ? desc->kernel : (zm ? 1 : 0);
    const bool packed = ctx->plan.packed;
    int tile = desc->tile >= 0 ? desc->tile : zmarch_default_tile(packed);
    if (ctx->kernel == 1 && desc->tile < 0 && !ctx->cache.empty()) {
        int t = zmarch_cache_lookup(ctx->cache.c_str(), ctx->lattice, ctx->precision,
                                    ctx->n_nodes, packed);
        if (t >= 0) tile = t;
    }
    if (zm) {
        st = set_tile(ctx, tile, nullptr, ctx->merge_rows);
        if (st != TAU1_OK) {
            delete ctx;
            return st;
        }
    } else {
        ctx->tile = tile;
    }
    *out = ctx;
    return TAU1_OK;
}

tau1_status tau1_step(tau1_ctx* ctx, int64_t nsteps) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    if (nsteps < 0) return TAU1_E_INVALID;
    if (nsteps >= ctx->graph_chunk) {
        if (!ctx->exec || ctx->graph_kernel != ctx->kernel || ctx->graph_tile != ctx->tile ||
            ctx->graph_parity != ctx->parity) {
            st = build_graph(ctx);
            if (st != TAU1_OK) return st;
        }
        while (nsteps >= ctx->graph_chunk) {
            HIP_TRY(hipGraphLaunch(ctx->exec, ctx->stream));
            nsteps -= ctx->graph_chunk;
            ctx->steps_done += ctx->graph_chunk;
        }
    }
    while (nsteps > 0) {
        st = launch_one(ctx, ctx->kernel, ctx->tile, ctx->parity);
        if (st != TAU1_OK) return st;
        ctx->parity ^= 1;
        --nsteps;
        ++ctx->steps_done;
    }
    return TAU1_OK;
}

tau1_status tau1_sync(tau1_ctx* ctx) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipGetLastError());
    return TAU1_OK;
}

}  // extern "C"

namespace {

tau1_status moments_impl(tau1_ctx* ctx, int32_t sample, double* r, double* u, bool phys_rho) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    if (sample < 0 || sample >= ctx->nsamples) return TAU1_E_INVALID;
    int nbad = 0;
    switch (ctx->precision) {
        case kF64: st = export_sample_t<kF64>(ctx, sample, r, u, &nbad, phys_rho); break;
        case kF32: st = export_sample_t<kF32>(ctx, sample, r, u, &nbad, phys_rho); break;
        case kF16: st = export_sample_t<kF16>(ctx, sample, r, u, &nbad, phys_rho); break;
        case kBF16: st = export_sample_t<kBF16>(ctx, sample, r, u, &nbad, phys_rho); break;
    }
    if (st != TAU1_OK) return st;
    return nbad ? TAU1_E_NONFINITE : TAU1_OK;
}

}  // namespace

extern "C" {

tau1_status tau1_moments(tau1_ctx* ctx, int32_t sample, double* rho, double* u) {
    return moments_impl(ctx, sample, rho, u, true);
}

tau1_status tau1_moments_drho(tau1_ctx* ctx, int32_t sample, double* drho, double* u) {
    return moments_impl(ctx, sample, drho, u, false);
}

tau1_status tau1_permeability(tau1_ctx* ctx, int32_t sample, int32_t axis, double* k,
                              double* mass) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    if (sample < 0 || sample >= ctx->nsamples || axis < 0 || axis > 2) return TAU1_E_INVALID;
    if (k && ctx->g[axis] == 0.0) return TAU1_E_INVALID;
    double res[4] = {0, 0, 0, 0};
    st = reduce_ws(ctx, sample, axis, res);
    if (st != TAU1_OK) return st;
    if (res[3] != 0.0 || !std::isfinite(res[0]) || !std::isfinite(res[1]))
        return TAU1_E_NONFINITE;
    if (k) *k = res[1];
    if (mass) *mass = res[0];
    return TAU1_OK;
}

tau1_status tau1_permeability_noalloc(tau1_ctx* ctx, int32_t sample, int32_t axis,
                                      double* out) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    if (sample < 0 || sample >= ctx->nsamples || axis < 0 || axis > 2) return TAU1_E_INVALID;
    if (!out || reinterpret_cast<uintptr_t>(out) % alignof(double) != 0) return TAU1_E_INVALID;
    if (!ctx->scratch) return TAU1_E_HIP;  // the device copy of `scratch` was not found
    // the partial count is fixed (kReduceBlocks), so every sample fits
    static_assert(kReduceBlocks * 4 <= kScratchDoubles, "scratch holds every partial");
    // every partial is written before the final pass reads it, so nothing is
    // cleared; the final pass writes the four results straight to `out`
    return reduce_launch(ctx, sample, axis, ctx->scratch, out);
}

tau1_status tau1_autotune(tau1_ctx* ctx, int32_t trial_steps) {
    tau1_status st = check_usable(ctx);
    if (st != TAU1_OK) return st;
    if (trial_steps < 1) return TAU1_E_INVALID;
    if (!zmarch_eligible(ctx)) return TAU1_OK;  // only the gather kernel applies
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // each lane layout's launch is timed alone at every tile: the layouts of
    // a batch (rows of different lengths, samples of different depths) may
    // prefer different z-segments
    std::vector<float> best_v(kNumVariants, 1e30f);
    std::vector<int> tile_v(kNumVariants, -1);
    float best = 1e30f;
    int best_tile = ctx->tile;
    for (int i = 0; i < kNumTiles && st == TAU1_OK; ++i) {
        // the chunk tile first: its launches load the card less than the
        // z-march's, and a card that has just run lighter launches runs the
        // next heavy ones at a transiently higher, then lower clock; ending
        // with the z-march tiles leaves it as the usual choice runs it
        const int t = i == 0 ? kChunkTile : i - 1;
        if (!zmarch_tile_ok(ctx->precision, ctx->plan.packed, t)) continue;
        if (t == kChunkTile && !any_chunks(ctx)) continue;
        st = set_tile(ctx, t);  // layouts timed alone, also where they share a launch
        if (st != TAU1_OK) break;
        float total = 0.0f;
        for (int g = 0; g < (int)ctx->zgroups.size() && st == TAU1_OK; ++g) {
            // the trial reads the current buffer and writes the spare one only
            st = launch_group(ctx, g, ctx->parity);
            if (st != TAU1_OK) break;
            HIP_TRY(hipEventRecord(e0, ctx->stream));
            for (int i = 0; i < trial_steps && st == TAU1_OK; ++i)
                st = launch_group(ctx, g, ctx->parity);
            HIP_TRY(hipEventRecord(e1, ctx->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            total += ms;
            const int v = ctx->zgroups[g].variant;
            // a layout without the chunk records runs a z-march tile in place
            // of the chunk tile: not a choice of its own
            if (t == kChunkTile && !ctx->zgroups[g].chunks) continue;
            if (ms < best_v[v]) {
                best_v[v] = ms;
                tile_v[v] = t;
            }
        }
        if (st == TAU1_OK && total < best) {
            best = total;
            best_tile = t;
        }
    }
    // the one launch of a batch's one-chunk rows runs every layout at the
    // occupancy of the widest, where the tiles each layout prefers alone need
    // not be the best: its whole step is timed with those tiles and with each
    // z-march tile for every layout, and the fastest is kept
    int merged_tile = -1;  // -1: the per-layout tiles
    if (st == TAU1_OK && ctx->merge_rows) {
        ctx->kernel = 1;
        float best_m = 1e30f;
        for (int t = -1; t < kNumTiles && st == TAU1_OK; ++t) {
            if (t >= 0 && (t == kChunkTile || !zmarch_tile_ok(ctx->precision, ctx->plan.packed, t)))
                continue;
            st = t < 0 ? set_tile(ctx, best_tile, tile_v.data(), true) : set_tile(ctx, t, nullptr, true);
            if (st != TAU1_OK) break;
            st = launch_one(ctx, 1, ctx->tile, ctx->parity);
            if (st != TAU1_OK) break;
            HIP_TRY(hipEventRecord(e0, ctx->stream));
            for (int i = 0; i < trial_steps && st == TAU1_OK; ++i)
                st = launch_one(ctx, 1, ctx->tile, ctx->parity);
            HIP_TRY(hipEventRecord(e1, ctx->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_m) {
                best_m = ms;
                merged_tile = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TAU1_OK) return st;
    ctx->kernel = 1;
    st = merged_tile >= 0 ? set_tile(ctx, merged_tile, nullptr, true)
                          : set_tile(ctx, best_tile, tile_v.data(), ctx->merge_rows);
    if (st != TAU1_OK) return st;
    // the cache keeps one tile per size bucket: the best single tile
    if (!ctx->cache.empty())
        zmarch_cache_store(ctx->cache.c_str(), ctx->lattice, ctx->precision, ctx->n_nodes,
                           best_tile, best / trial_steps);
    return TAU1_OK;
}

tau1_status tau1_get_info(const tau1_ctx* ctx, tau1_info* info) {
    if (!ctx || !info) return TAU1_E_INVALID;
    info->lattice = ctx->lattice;
    info->precision = ctx->precision;
    info->n_samples = ctx->nsamples;
    info->kernel = ctx->kernel;
    info->tile = ctx->tile;
    info->graph_chunk = ctx->graph_chunk;
    info->layout = ctx->plan.packed ? 1 : 0;
    info->n_nodes = ctx->n_nodes;
    info->n_fluid = ctx->n_fluid;
    info->steps_done = ctx->steps_done;
    const double s = storage_bytes(ctx->precision);
    const double vals = ctx->lattice == 9 ? 3.0 : 4.0;  // d + 1 stored values per node
    info->bytes_per_step = 2.0 * vals * s * (double)ctx->n_fluid + (double)ctx->n_nodes / 8.0;
    int64_t items = 0;
    if (ctx->kernel == 1)
        for (const auto& g : ctx->zgroups) items += g.args[0].ntiles;
    info->work_items = items;
    int launches = 0;
    for (int g = 0; g < launch_groups(ctx, ctx->kernel); ++g)
        if (step_launch(ctx, ctx->kernel, ctx->tile, g).grid.x > 0) ++launches;
    info->launches_per_step = launches;
    return TAU1_OK;
}

void tau1_destroy(tau1_ctx* ctx) {
    if (!ctx) return;
    destroy_graph(ctx);
    delete ctx;
}

tau1_status tau1_copy_probe(void* hip_stream, void* buf, size_t bytes, int32_t reps,
                            double* seconds) {
    if (!buf || bytes < 64 || reps < 1 || !seconds) return TAU1_E_INVALID;
    tau1_ctx* ctx = nullptr;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t n = (int64_t)(bytes / 2 / 16);
    const float4* src = reinterpret_cast<const float4*>(buf);
    float4* dst = reinterpret_cast<float4*>(reinterpret_cast<uint8_t*>(buf) + n * 16);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)1 << 22);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, stream, src, dst, n);
    HIP_TRY(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, stream, src, dst, n);
    HIP_TRY(hipEventRecord(e1, stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *seconds = ms * 1e-3 / reps;
    return TAU1_OK;
}

}  // extern "C"
