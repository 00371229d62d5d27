// One (BATCH, EDGE, RULE) combination of the edge-record step's launchers,
// chosen by NBB_INST_BATCH (0/1), NBB_INST_EDGE (0/1) and NBB_INST_RULE (0:
// B3/S23, 1: table look-up, 2: bit extract); the build compiles this file
// once per combination.
#include "edges.hpp"
#include "edges_launch.hpp"

#if !defined(NBB_INST_BATCH) || !defined(NBB_INST_EDGE) || !defined(NBB_INST_RULE)
#error "edges_inst.hip needs NBB_INST_BATCH, NBB_INST_EDGE and NBB_INST_RULE"
#endif

namespace nbb {

template <bool BATCH, bool EDGE, int RULE>
hipError_t launch_edges_inst(const EdgeParams &E, uint32_t BS, uint32_t nsrc, const uint8_t *in, uint8_t *out,
                             uint32_t rule, const uint32_t *rec, int cu_count, EdgeCaps caps, hipStream_t st) {
    return launch_edges_shape<BATCH, EDGE, RULE>(E, BS, nsrc, in, out, rule, rec, cu_count, caps, st);
}

template hipError_t launch_edges_inst<bool(NBB_INST_BATCH), bool(NBB_INST_EDGE), NBB_INST_RULE>(
    const EdgeParams &, uint32_t, uint32_t, const uint8_t *, uint8_t *, uint32_t, const uint32_t *, int, EdgeCaps,
    hipStream_t);

}  // namespace nbb
