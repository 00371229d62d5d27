// One (BATCH, TEAM, EDGE) combination of the tiled step's launchers, chosen by
// NBB_INST_BATCH (0/1), NBB_INST_TEAM (64/256) and NBB_INST_EDGE (0/1); the
// build compiles this file once per combination.
#include "tiled.hpp"
#include "tiled_launch.hpp"

#if !defined(NBB_INST_BATCH) || !defined(NBB_INST_TEAM) || !defined(NBB_INST_EDGE)
#error "tiled_inst.hip needs NBB_INST_BATCH, NBB_INST_TEAM and NBB_INST_EDGE"
#endif

namespace nbb {

template <bool BATCH, int TEAM, bool EDGE>
hipError_t launch_tiled_inst(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                             uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    return launch_tiled_bs<BATCH, TEAM, EDGE>(P, T, in, out, rule, rec, cu_count, st);
}

template hipError_t launch_tiled_inst<bool(NBB_INST_BATCH), NBB_INST_TEAM, bool(NBB_INST_EDGE)>(
    const MapParams &, const TileParams &, const uint8_t *, uint8_t *, uint32_t, const uint32_t *, int, hipStream_t);

}  // namespace nbb
