// tau1_zmarch_inst.hip -- instantiates the z-march kernels and the chunk
// kernels of one (lattice, precision) pair, chosen with -DTAU1_Q=.. -DTAU1_P=..
// at build time, so the pairs compile in parallel.
#include "tau1_chunks.hpp"

#ifndef TAU1_Q
#error "TAU1_Q must be defined"
#endif
#ifndef TAU1_P
#error "TAU1_P must be defined"
#endif

namespace tau1 {

#define TAU1_CAT2(a, b, c) a##b##_##c
#define TAU1_CAT(a, b, c) TAU1_CAT2(a, b, c)

// Kernel of layout V for load mode 0-3; modes 1 and 3 on a multi-row layout
// are mode 2's schedule at two waves per SIMD and share one instance.
template <int V>
void* zm_pick(int mode) {
    if (mode == 0) return reinterpret_cast<void*>(&k_zmarch<TAU1_Q, TAU1_P, V, 0>);
    if constexpr (kVariants[V].g == 1) {
        if (mode == 1) return reinterpret_cast<void*>(&k_zmarch<TAU1_Q, TAU1_P, V, 1>);
        if (mode == 3) return reinterpret_cast<void*>(&k_zmarch<TAU1_Q, TAU1_P, V, 3>);
    } else {
        if (mode == 1 || mode == 3) return reinterpret_cast<void*>(&k_zmarch<TAU1_Q, TAU1_P, V, 1>);
    }
    return reinterpret_cast<void*>(&k_zmarch<TAU1_Q, TAU1_P, V, 2>);
}

void* TAU1_CAT(zm_kernel_, TAU1_Q, TAU1_P)(int variant, int mode) {
    if (mode < 0 || mode > 3) return nullptr;
    switch (variant) {
#define TAU1_V(V) case V: return zm_pick<V>(mode);
        TAU1_V(0) TAU1_V(1) TAU1_V(2) TAU1_V(3) TAU1_V(4) TAU1_V(5) TAU1_V(6) TAU1_V(7)
        TAU1_V(8) TAU1_V(9) TAU1_V(10) TAU1_V(11) TAU1_V(12) TAU1_V(13) TAU1_V(14)
#undef TAU1_V
    }
    return nullptr;
}

// Chunk kernel for lane chunks of K nodes (the packed layouts use K = 1..6).
void* TAU1_CAT(ck_kernel_, TAU1_Q, TAU1_P)(int k) {
    switch (k) {
        case 1: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 1>);
        case 2: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 2>);
        case 3: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 3>);
        case 4: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 4>);
        case 5: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 5>);
        case 6: return reinterpret_cast<void*>(&k_chunks<TAU1_Q, TAU1_P, 6>);
    }
    return nullptr;
}

}  // namespace tau1
