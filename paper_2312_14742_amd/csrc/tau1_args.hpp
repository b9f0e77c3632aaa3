// tau1_args.hpp -- launch arguments shared by every step kernel (the z-march
// tiles, the per-node gather, the D2Q9 kernel) and the service kernels, with
// the storage-scale accessors the kernels read them through.
#pragma once

#include "tau1_device.hpp"

namespace tau1 {

// Arguments shared by every step kernel (passed by value; one copy per
// ping-pong parity is kept by the host so HIP graph nodes can point at it).
struct StepArgs {
    uint8_t* base;              // workspace base
    const SampleDev* samples;   // device array, nsamples entries
    const int32_t* tiles;       // z-march work list (sample, ty, tz) triples
    int32_t nsamples;
    int32_t parity;             // buffer read this step; the other is written
    int32_t ntiles;             // z-march work items
    int32_t pad;
    double gh[3];               // g / 2 (FP64)
    float ghf[3];               // g / 2 (FP32)
    float scale_rho, inv_scale_rho, scale_u, inv_scale_u;  // F16 storage
    // D2Q9 boundaries: Zou-He pressure columns at x = 0 and nx - 1 (xbc = 1)
    // with densities 1 + din, 1 + dout; velocity of the moving walls
    int32_t xbc;
    int32_t pad2;
    double din, dout;
    double uw[2];
};

template <int P>
__device__ __forceinline__ typename Storage<P>::T inv_scale_rho(const StepArgs& a) {
    if constexpr (P == kF16) return a.inv_scale_rho; else return 1;
}
template <int P>
__device__ __forceinline__ typename Storage<P>::T inv_scale_u(const StepArgs& a) {
    if constexpr (P == kF16) return a.inv_scale_u; else return 1;
}
template <int P>
__device__ __forceinline__ typename Storage<P>::T scale_rho(const StepArgs& a) {
    if constexpr (P == kF16) return a.scale_rho; else return 1;
}
template <int P>
__device__ __forceinline__ typename Storage<P>::T scale_u(const StepArgs& a) {
    if constexpr (P == kF16) return a.scale_u; else return 1;
}
template <typename T>
__device__ __forceinline__ T gh_of(const StepArgs& a, int d) {
    if constexpr (sizeof(T) == 8) return a.gh[d]; else return a.ghf[d];
}

}  // namespace tau1
