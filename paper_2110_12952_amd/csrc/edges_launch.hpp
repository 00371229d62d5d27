// Entry to the edge-record step's launchers, one per (BATCH, EDGE, RULE),
// each defined in its own build of edges_inst.hip.  RULE 0 = B3/S23 (Moore
// only), 1 = a rule without birth or survival at 8, 2 = any Moore rule.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.hpp"

namespace nbb {

template <bool BATCH, bool EDGE, int RULE>
hipError_t launch_edges_inst(const EdgeParams &E, uint32_t BS, uint32_t nsrc, const uint8_t *in, uint8_t *out,
                             uint32_t rule, const uint32_t *rec, int cu_count, EdgeCaps caps, hipStream_t st);

#define NBB_EDGES_INST_DECL(B, E, R)                                                                       \
    extern template hipError_t launch_edges_inst<B, E, R>(const EdgeParams &, uint32_t, uint32_t,          \
                                                          const uint8_t *, uint8_t *, uint32_t,            \
                                                          const uint32_t *, int, EdgeCaps, hipStream_t);
NBB_EDGES_INST_DECL(false, false, 0)
NBB_EDGES_INST_DECL(false, false, 1)
NBB_EDGES_INST_DECL(false, false, 2)
NBB_EDGES_INST_DECL(false, true, 1)
NBB_EDGES_INST_DECL(true, false, 0)
NBB_EDGES_INST_DECL(true, false, 1)
NBB_EDGES_INST_DECL(true, false, 2)
NBB_EDGES_INST_DECL(true, true, 1)
#undef NBB_EDGES_INST_DECL

// The rule's form for the launchers above: 0 for B3/S23, 1 when no entry at
// eight neighbours is set (and always for the four-cell stencil), else 2.
inline int edges_rule_kind(uint32_t rule) {
    if (rule == ((1u << 3) | ((1u << 2 | 1u << 3) << 16))) return 0;
    if ((rule >> 31) || (rule & ((1u << 8) | (1u << 24))) == 0) return 1;
    return 2;
}

}  // namespace nbb
