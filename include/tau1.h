/*
 * tau1.h -- C ABI of the MI355X (gfx950) Tau1 lattice Boltzmann library.
 *
 * Method (Bacza, Tomczak, Matyka, "The lattice Boltzmann method for fluid
 * flows at relaxation time equal one: performance study"): with relaxation
 * time tau = 1 the LBGK update of Eq. (4) reduces to Eq. (8), so only the
 * density and velocity are stored (two copies, "AB" layout).  Each fluid node
 * gathers rho and u of its neighbours x - c_k, forms the equilibrium of
 * Eq. (3) for direction k and sums them into the new rho and momentum
 * (Eqs. (9)-(10)); the velocity is the momentum times one reciprocal of rho
 * (the division-saving algorithm of the implementation section).  Links to
 * solid nodes use halfway bounce-back with the population rebuilt from the
 * node's own previous rho*, u* (Eq. (11)).  All axes are periodic; walls are
 * solid nodes.  A body force g (an acceleration, lattice units) enters as a
 * velocity shift: the equilibrium is evaluated at u + g/2 and the reported
 * velocity is j/rho + g/2.
 *
 * Lattices D3Q15, D3Q19, D3Q27 (the 3-D sets of the complexity table).
 * Node index: x + nx*(y + ny*z), x fastest.  Every size is in nodes unless
 * stated.
 *
 * Memory: the library never allocates device memory.  The caller queries
 * tau1_workspace_size and passes a device buffer of at least that many bytes
 * (for example a torch uint8 tensor); the buffer and the HIP stream are
 * borrowed and must outlive the context.  The context owns only host-side
 * metadata and its HIP graphs.  Host arrays passed in are copied during the
 * call; host output arrays are written during the call.
 *
 * Errors: every call returns a tau1_status; no C++ exception crosses the ABI.
 * On error, output arguments are left untouched and a failed create leaves
 * *out == NULL.  TAU1_E_HIP is sticky: the context must be destroyed.
 * tau1_step only enqueues work; device faults surface at the next call that
 * synchronises (tau1_moments, tau1_permeability, tau1_sync).
 *
 * Threading: a context is not thread-safe; distinct contexts are independent.
 *
 * State layout (internal to the workspace; results are bit-for-bit the same
 * in both): "dense" stores every node; "packed" stores only the runs of K
 * consecutive x-nodes (the z-march lane chunks, K fixed by nx) that hold at
 * least one fluid node, so the state is smaller and a step moves fewer bytes.
 * Packing applies to the samples whose nx has a one-row-per-wave z-march
 * layout (nx = 64, 96, 128, 160, 192, 224, 256, 288, 320, 384, 512); the
 * other samples of the context stay dense.
 */
#ifndef TAU1_H
#define TAU1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TAU1_OK = 0,
    TAU1_E_INVALID = -1,     /* bad argument (dims, lattice, precision, ...) */
    TAU1_E_NOMEM = -2,       /* host allocation failed                       */
    TAU1_E_HIP = -3,         /* a HIP runtime call or kernel failed (sticky)  */
    TAU1_E_UNSUPPORTED = -4, /* valid request this build does not provide     */
    TAU1_E_NONFINITE = -5,   /* a reduction or readback met NaN or Inf        */
    TAU1_E_WORKSPACE = -6    /* workspace missing, too small or misaligned    */
} tau1_status;

typedef struct tau1_ctx tau1_ctx; /* opaque, owned by the library */

/* D2Q9 is the two-dimensional lattice of the paper's validation runs
 * (pressure-driven Poiseuille flow, lid-driven cavity): samples have nz = 1,
 * F64 or F32 only, one thread per node; its node types and boundaries are
 * described at tau1_desc. */
typedef enum { TAU1_D2Q9 = 9, TAU1_D3Q15 = 15, TAU1_D3Q19 = 19, TAU1_D3Q27 = 27 } tau1_lattice;

/* Arithmetic and storage of (rho - 1, u):
 *   TAU1_F64       FP64 compute, FP64 storage (parity mode);
 *   TAU1_F32       FP32 compute, FP32 storage;
 *   TAU1_F32_F16   FP32 compute, IEEE half storage with power-of-two scales;
 *   TAU1_F32_BF16  FP32 compute, bfloat16 storage (round to nearest even).
 * Mass and permeability are always reduced in FP64. */
typedef enum {
    TAU1_F64 = 0,
    TAU1_F32 = 1,
    TAU1_F32_F16 = 2,
    TAU1_F32_BF16 = 3
} tau1_precision;

/* One lattice (one porous sample). */
typedef struct {
    int64_t nx, ny, nz;    /* >= 1 each; every axis periodic                  */
    const uint8_t *solid;  /* host, N bytes; nonzero = solid node              */
    const double *drho0;   /* host, N values of rho - 1, or NULL for rho = 1   */
    const double *u0;      /* host, 3N values, SoA (ux | uy | uz), or NULL     */
} tau1_sample;

typedef struct {
    int32_t lattice;        /* tau1_lattice                                    */
    int32_t precision;      /* tau1_precision                                  */
    int32_t n_samples;      /* >= 1; > 1 = batched: the samples of one lane
                               layout (row length nx) share one kernel launch
                               per step, each layout its own launch         */
    int32_t graph_chunk;    /* steps per captured HIP graph; even; 0 = 100      */
    const tau1_sample *samples;
    double g[3];            /* body acceleration, same for every sample         */
    void *hip_stream;       /* borrowed hipStream_t; NULL = default stream      */
    void *workspace;        /* borrowed device memory, 256-byte aligned         */
    size_t workspace_bytes;
    int32_t kernel;         /* step kernel: -1 = automatic (tuned or default),
                               0 = per-node gather, 1 = z-march tiles        */
    int32_t tile;           /* z-march tile shape, -1 = automatic; 0-15 =
                               z-segment of 16/32/64/128 planes (tile % 4) x
                               load schedule (tile / 4: 0 just in time,
                               1 rows shared through LDS, 2 rolling prefetch,
                               3 shared rows on the packed layout); 16 = one
                               lane per stored chunk instead of a z-march
                               (for rows that are mostly solid; same bits);
                               a packed context takes 12-16, a dense one 0-11 */
    int32_t f16_log2_scale_rho; /* F16 storage: stored = value * 2^s; 0 = 16.
                                   Half holds |value| < 65504 * 2^-s (0.9995
                                   at s = 16) and is normal down to 2^-(14+s)
                                   (9.3e-10 at s = 16); tau1_create rejects an
                                   initial |rho - 1| above half that range
                                   (TAU1_E_INVALID), and a state that grows
                                   past it later reads back as Inf
                                   (TAU1_E_NONFINITE from tau1_moments and
                                   tau1_permeability)                       */
    int32_t f16_log2_scale_u;   /* F16 scale of the stored velocity u + g/2,
                                   0 = 16; same range and check as above    */
    const char *tune_cache; /* path of the autotune JSON cache, or NULL         */
    int32_t layout;         /* state layout: -1 = automatic (packed for F32,
                               F16 and BF16 z-march contexts unless tile is
                               0-11, dense otherwise), 0 = dense, 1 = packed
                               (TAU1_E_UNSUPPORTED if no sample can be
                               packed: F64, kernel 0, other nx)            */
    /* D2Q9 only (TAU1_E_UNSUPPORTED on the 3-D lattices when set).  Solid
     * bytes there are node types: 0 fluid, 1 wall (halfway bounce-back),
     * 2 moving wall (bounce-back plus the wall momentum 6 w_k rho (c_k . u_w)).
     * g[2] must be 0; the z component of u0 is ignored.                   */
    int32_t x_boundary;     /* 0 = periodic in x; 1 = constant-pressure
                               (Zou-He) columns: fluid nodes at x = 0 hold
                               rho_in, at x = nx - 1 rho_out (nx >= 3)      */
    double rho_in, rho_out; /* > 0, used when x_boundary = 1              */
    double wall_u[3];       /* velocity of the moving walls (z ignored)    */
    /* Launch and graph shape of a batch whose samples have several lane
     * layouts (rows of different lengths; one z-march launch per layout):
     * 1 = one chain: the launches of a step run one after another, largest
     * first, each with the whole GPU; 2 = one chain per lane layout, the
     * chains running side by side; 3 = one launch per step for every sample
     * whose row is 64-320 nodes long (one lane chunk per row) and whose tile
     * runs the rows-shared-through-LDS schedule of the leading such layout
     * (the others, such as rows of 384 or 512 nodes, launch alone, in
     * chains as with 2); the results are the same bits in every shape;
     * 0 = automatic (2, measured the faster on the 64-sample batch).
     * Single-launch contexts ignore it; values outside 0-3 are
     * TAU1_E_INVALID.                                                        */
    int32_t batch_graph;
} tau1_desc;

/* Static facts about a created context (host copy). */
typedef struct {
    int32_t lattice, precision, n_samples;
    int32_t kernel;          /* step kernel in use: 0 per-node gather,
                                1 z-march tiles, 2 D2Q9                     */
    int32_t tile;            /* tile in use (z-march tiles and the chunk
                                tile); in a batch, that of the lane layout
                                with the most fluid nodes (tau1_autotune
                                gives each layout its own)                 */
    int32_t graph_chunk;
    int32_t layout;          /* 1 if any sample is stored packed, else 0    */
    int64_t n_nodes;         /* all samples                                 */
    int64_t n_fluid;         /* all samples                                 */
    int64_t steps_done;
    double bytes_per_step;   /* algorithmic HBM bytes of one step (all samples):
                                2 (d+1) s per fluid node plus one mask bit per
                                node (complexity table of the paper)        */
    int64_t work_items;      /* work items per step: z-march row groups x
                                z-segments holding a fluid node, or waves of
                                64 stored chunks for the chunk tile; 0 for
                                the gather kernel                           */
    int32_t launches_per_step; /* kernel launches one step takes (one per
                                z-march lane layout, or one for all the
                                one-chunk rows with batch_graph 3)          */
} tau1_info;

/* Bytes of device workspace the descriptor needs: two copies of the state
 * (the "AB" layout of the Tau1 algorithm, Section 2.1; d + 1 values per node,
 * complexity table of Section 2.1.3) plus the geometry tables.  Host only, no
 * GPU call.  *bytes is written only on TAU1_OK. */
tau1_status tau1_workspace_size(const tau1_desc *desc, size_t *bytes);

/* Validates the descriptor, encodes the geometry (the node types of Section
 * 2.1.3: a bit mask, the wall-node lists for bounce-back, the packed chunk
 * table) and uploads the initial rho - 1 and u into the workspace (both
 * copies).  Host arrays are read during the call only.  Synchronous on the
 * stream.  TAU1_E_INVALID for a bad descriptor or initial field (non-finite,
 * rho <= 0, or outside the F16 range), TAU1_E_WORKSPACE for a missing,
 * misaligned or too small workspace, TAU1_E_UNSUPPORTED for a valid request
 * this build does not serve.  On error *out is NULL and nothing is owned. */
tau1_status tau1_create(const tau1_desc *desc, tau1_ctx **out);

/* Enqueues nsteps >= 0 time steps on the stream and returns without waiting
 * (graph replays of graph_chunk steps, then single launches).  One step
 * advances every fluid node of every sample by the Tau1 update: the
 * equilibria of Eq. (3) at the sources x - c_k arrive at x (Eq. (8)), their
 * zeroth and first moments are the new density and momentum (Eqs. (9)-(10),
 * Section 2.1), the velocity is the momentum times one reciprocal of the
 * density (Section 3, division-saving algorithm), and a link whose source is
 * solid returns the node's own previous equilibrium in the opposite direction
 * (halfway bounce-back, Eq. (11), Section 2.1.1).  Device errors surface at
 * the next synchronising call. */
tau1_status tau1_step(tau1_ctx *ctx, int64_t nsteps);

/* Waits for the stream and reports any pending device error. */
tau1_status tau1_sync(tau1_ctx *ctx);

/* Copies the current state of one sample to host FP64 arrays: rho (N values,
 * the physical density of Eq. (9), rho = 1 + (rho - 1) formed in FP64) and
 * u (3N values, SoA, the velocity of Eq. (10) divided by rho, including the
 * g/2 shift of the forcing).  Solid nodes read rho = 1, u = 0.  Either
 * pointer may be NULL.  Synchronous.  TAU1_E_NONFINITE if any fluid value is
 * NaN or Inf (the arrays are still written); TAU1_E_INVALID for a sample out
 * of range. */
tau1_status tau1_moments(tau1_ctx *ctx, int32_t sample, double *rho, double *u);

/* As tau1_moments, but the first array receives rho - 1 exactly as the state
 * holds it (the library stores the density as rho - 1, which keeps the
 * small density variations of Eq. (9) at full precision; solid nodes read 0).
 * Restarting from a saved state passes this array as drho0. */
tau1_status tau1_moments_drho(tau1_ctx *ctx, int32_t sample, double *drho,
                              double *u);

/* FP64 reductions over one sample, in a fixed order (deterministic):
 *   mass = sum over fluid nodes of rho (Eq. (5); conserved by the update);
 *   k    = nu <u_axis> / g_axis, nu = 1/6, <.> the mean over all N nodes
 *          (Darcy permeability in lattice units; solid nodes count as 0).
 * The paper defines no permeability: this is Darcy's law with the kinematic
 * viscosity of tau = 1, nu = (tau - 1/2)/3 = 1/6.  k may be NULL; if it is
 * not, g[axis] must be nonzero (TAU1_E_INVALID).  Synchronous.
 * TAU1_E_NONFINITE if a fluid node holds NaN or Inf (outputs untouched). */
tau1_status tau1_permeability(tau1_ctx *ctx, int32_t sample,
                              int32_t axis, double *k, double *mass);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): the reductions of
 * tau1_permeability, enqueued on the context's stream without waiting.  The
 * block partials live in a static device array of this library (32 KiB per
 * GPU, held until the process ends; it serves every sample size, since the
 * partial count is fixed), so the call allocates nothing, sets no memory and
 * copies nothing to the host.  out: caller-owned device memory of 4 doubles,
 * 8-byte aligned, written when the stream reaches the call: out[0] = mass,
 * out[1] = k (0 when g[axis] == 0), out[2] = fluid node count, out[3] =
 * count of fluid nodes holding NaN or Inf.  Results are bit-for-bit those of
 * tau1_permeability.  Calls on one GPU share the array: calls that overlap in
 * time on that GPU (other streams, other threads) race and must not be
 * issued.  TAU1_E_INVALID for a bad sample, axis or out; TAU1_E_HIP if the
 * array's device address could not be found. */
tau1_status tau1_permeability_noalloc(tau1_ctx *ctx, int32_t sample,
                                      int32_t axis, double *out);

/* Times each eligible step-kernel shape for trial_steps steps (state is not
 * advanced: trials write only the spare buffer), keeps the fastest and, if
 * the descriptor named a cache file, records it there.  In a batch each lane
 * layout is timed alone and gets its own tile; with batch_graph 3 the whole
 * step is then timed with those tiles and with each z-march tile for every
 * layout, and the fastest is kept.  Synchronous.  An engineering aid of this
 * library (the paper tunes thread counts by hand, Section 4). */
tau1_status tau1_autotune(tau1_ctx *ctx, int32_t trial_steps);

/* Static facts about the context (host copy); bytes_per_step is the
 * complexity table's 2 (d+1) s bytes per fluid node plus one mask bit per
 * node (Section 2.1.3). */
tau1_status tau1_get_info(const tau1_ctx *ctx, tau1_info *info);

/* Releases host resources (graphs, metadata); NULL-safe. */
void tau1_destroy(tau1_ctx *ctx);

const char *tau1_strerror(tau1_status status);

/* Copy-bandwidth probe (calibrates the achievable HBM rate, the GPU analogue
 * of the copy loop the paper measures against in Section 4.2): copies
 * bytes/2 from the first half of buf to the second half, reps times, on the
 * stream; returns the mean seconds per copy measured with HIP events.  buf is
 * device memory of at least `bytes`, borrowed for the call. */
tau1_status tau1_copy_probe(void *hip_stream, void *buf, size_t bytes,
                            int32_t reps, double *seconds);

#ifdef __cplusplus
}
#endif
#endif /* TAU1_H */
