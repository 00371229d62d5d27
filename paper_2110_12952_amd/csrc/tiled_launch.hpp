// Entry to the tiled step's launchers, one per (BATCH, TEAM, EDGE).  Each is
// defined in its own build of tiled_inst.hip (NBB_INST_BATCH, NBB_INST_TEAM,
// NBB_INST_EDGE), so the instantiations compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.hpp"

namespace nbb {

template <bool BATCH, int TEAM, bool EDGE>
hipError_t launch_tiled_inst(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                             uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st);

#define NBB_TILED_INST_DECL(B, T, E)                                                                          \
    extern template hipError_t launch_tiled_inst<B, T, E>(const MapParams &, const TileParams &, const uint8_t *, \
                                                          uint8_t *, uint32_t, const uint32_t *, int, hipStream_t);
NBB_TILED_INST_DECL(false, 64, false)
NBB_TILED_INST_DECL(false, 64, true)
NBB_TILED_INST_DECL(false, 256, false)
NBB_TILED_INST_DECL(false, 256, true)
NBB_TILED_INST_DECL(true, 64, false)
NBB_TILED_INST_DECL(true, 64, true)
NBB_TILED_INST_DECL(true, 256, false)
NBB_TILED_INST_DECL(true, 256, true)
#undef NBB_TILED_INST_DECL

}  // namespace nbb
