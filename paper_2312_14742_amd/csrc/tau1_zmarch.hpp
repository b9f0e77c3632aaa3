// tau1_zmarch.hpp -- z-march tiled step kernel (placeholder: not yet built).
#pragma once
#include <vector>
#include "tau1_kernels.hpp"

namespace tau1 {
constexpr int kNumTiles = 1;
inline void zmarch_tiling(SampleDev& sd) { sd.tiles_y = 0; sd.tiles_z = 0; }
inline bool zmarch_supported(int, int, const void*, int) { return false; }
inline bool zmarch_tile_ok(int, int, int) { return false; }
inline void* pick_zmarch(int, int, int) { return nullptr; }
inline int zmarch_threads(int) { return 64; }
inline int64_t zmarch_grid(int64_t, int) { return 0; }
template <typename SH>
inline std::vector<int32_t> zmarch_worklist(const SH*, int, int64_t) { return {}; }
inline int zmarch_default_tile(int, int) { return 0; }
inline int zmarch_cache_lookup(const char*, int, int, int64_t) { return -1; }
inline void zmarch_cache_store(const char*, int, int, int64_t, int, float) {}
}  // namespace tau1
