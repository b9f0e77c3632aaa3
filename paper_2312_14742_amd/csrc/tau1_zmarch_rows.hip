// tau1_zmarch_rows.hip -- instantiates the one-launch z-march kernels (every
// one-row lane layout of a batch in one launch) of one (lattice, precision)
// pair, chosen with -DTAU1_Q=.. -DTAU1_P=.. at build time.
#include "tau1_zmarch.hpp"

#ifndef TAU1_Q
#error "TAU1_Q must be defined"
#endif
#ifndef TAU1_P
#error "TAU1_P must be defined"
#endif

namespace tau1 {

#define TAU1_CAT2(a, b, c) a##b##_##c
#define TAU1_CAT(a, b, c) TAU1_CAT2(a, b, c)

// Mode 1 (dense rows shared through LDS) or 3 (packed rows shared through LDS).
void* TAU1_CAT(zr_rows_kernel_, TAU1_Q, TAU1_P)(int mode) {
    if (mode == 1) return reinterpret_cast<void*>(&k_zmarch_rows<TAU1_Q, TAU1_P, 1>);
    if (mode == 3) return reinterpret_cast<void*>(&k_zmarch_rows<TAU1_Q, TAU1_P, 3>);
    return nullptr;
}

}  // namespace tau1
