// Host launchers for the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.hpp"

namespace nbb {

hipError_t launch_lambda(const MapParams &P, uint32_t lam_words, const uint32_t *idx, uint64_t count,
                         int32_t *x, int32_t *y, int grid, hipStream_t st);
hipError_t launch_lambda_digits(const MapParams &P, const uint32_t *idx, uint64_t count, int32_t *x, int32_t *y,
                                int grid, hipStream_t st);
hipError_t launch_nu_digits(const MapParams &P, const int32_t *x, const int32_t *y, uint64_t count, uint32_t *idx,
                            int grid, hipStream_t st);
hipError_t launch_lambda_mfma(const MapParams &P, const MfmaLambda &M, const uint32_t *idx, uint64_t count,
                              int32_t *x, int32_t *y, int grid, hipStream_t st);
hipError_t launch_nu_mfma(const MapParams &P, const MfmaLambda &M, const int32_t *x, const int32_t *y, uint64_t count,
                          uint32_t *idx, int grid, hipStream_t st);
hipError_t launch_nu(const MapParams &P, uint32_t nu_halves, const int32_t *x, const int32_t *y,
                     uint64_t count, uint32_t *idx, int grid, hipStream_t st);
hipError_t launch_init_compact(const MapParams &P, uint32_t lam_words, uint8_t *state, uint64_t seed,
                               uint32_t thr, int grid, hipStream_t st);
hipError_t launch_init_box(const BoxParams &B, uint8_t *state, uint64_t seed, uint32_t thr, hipStream_t st);
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t st);   // bytes / 16 chunks; p 16-aligned
hipError_t launch_fill_tail(void *p, uint32_t bytes, hipStream_t st);   // bytes < 64, any alignment
hipError_t launch_expand(const MapParams &P, uint32_t lam_words, const uint8_t *compact, uint8_t *box,
                         uint64_t pitch, int grid, hipStream_t st);
hipError_t launch_gather(const MapParams &P, uint32_t lam_words, const uint8_t *box, uint64_t pitch,
                         uint8_t *compact, int grid, hipStream_t st);
hipError_t launch_step_direct(const MapParams &P, uint32_t lam_words, uint32_t nu_halves, const uint8_t *in,
                              uint8_t *out, uint32_t rule, int grid, hipStream_t st);
hipError_t launch_blocked_scatter(const TileParams &T, const uint8_t *compact, uint8_t *blocked, uint64_t cells,
                                  int grid, hipStream_t st);
hipError_t launch_blocked_gather(const TileParams &T, const uint8_t *blocked, uint8_t *compact, uint64_t cells,
                                 int grid, hipStream_t st);
hipError_t launch_step_blocked(const TileParams &T, const uint8_t *in, uint8_t *out, uint32_t rule, int cu_count,
                               hipStream_t st);
hipError_t launch_step_lambda(const MapParams &P, uint32_t lam_words, const uint8_t *in, uint8_t *out,
                              uint64_t pitch, uint32_t rule, int grid, hipStream_t st);
// Persistent launch sized to the resident capacity of cu_count CUs.
hipError_t launch_step_tiled(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                             uint32_t rule, int cu_count, hipStream_t st);
// The tiled step in edge-record form (edges.hpp): BS 3 or 4, nsrc 2 or 4
// source dwords per block; rec = NULL for one instance, else the batch's
// per-tile records (E.nbr / E.ntiles then the batch's).  limit: bytes of
// `in` the step may read (the state's k^r, or the arena's length).
hipError_t launch_step_edges(const EdgeParams &E, uint32_t BS, uint32_t nsrc, const uint8_t *in, uint8_t *out,
                             uint64_t limit, uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st);
// The tiled step over the tiles of a batch (tables from launch_batch_tiles,
// T.ntiles = batch tiles, T.nbr = the batch neighbour table).
hipError_t launch_step_tiled_batch(const TileParams &T, const uint32_t *rec, const uint8_t *arena_in,
                                   uint8_t *arena_out, uint32_t rule, int cu_count, hipStream_t st);
// LDS bytes the LDS-resident batch step needs for an instance of `ntiles`
// tiles of plan T stepped by `teams` tiles at a time (boxes, two state
// copies, neighbour table).
uint32_t resident_lds_bytes(const TileParams &T, uint32_t ntiles, uint32_t teams);
// Whether a tile of plan T fits the per-thread registers of the resident step
// when a work-group works on `teams` (1, 2 or 4) tiles at a time.
bool resident_fits(const TileParams &T, uint32_t teams);
// All generations of `count` small instances, one work-group each (inst:
// device table; plans: device table of the plans inst[w].plan indexes, each
// checked with resident_fits for its instances' teams; instance w takes
// steps_of[w] generations, a device array, or steps_all if steps_of is NULL;
// lds = the largest resident_lds_bytes).  Instance w's result ends in a if
// its generation count is even, else in b.
hipError_t launch_step_resident(const TileParams *plans, const ResidentInstance *inst, uint32_t count,
                                const uint32_t *steps_of, uint32_t steps_all, uint32_t lds, uint8_t *a, uint8_t *b,
                                uint32_t rule, hipStream_t st);
// Stores n host words at dst (device) in stream order, through kernels that
// take them as arguments (no host memory is read after the call returns).
hipError_t launch_set_words(uint32_t *dst, const uint32_t *src, uint32_t n, hipStream_t st);
// Builds the per-tile record and neighbour tables of a batch on the device.
hipError_t launch_batch_tiles(const BatchInstance *inst, uint32_t ninst, uint32_t total, uint32_t *rec,
                              uint32_t *nbr, hipStream_t st);
// `gens` <= T.h generations of every tile of a temporal plan in one launch
// (temporal.hip); one work-group per tile.
hipError_t launch_step_temporal(const TemporalParams &T, const uint8_t *in, uint8_t *out, uint32_t rule,
                                uint32_t gens, hipStream_t st);
hipError_t launch_step_box(const BoxParams &B, const uint8_t *in, uint8_t *out, uint32_t rule, hipStream_t st);
// Bit-packed compact state (cell i = bit i % 32 of word i / 32): conversions
// from and to one byte per cell (any non-zero byte packs as 1; words past the
// last cell hold zero bits), and the tiled step on it.  lutw: 32 phase copies
// of the plan's lut0, `stride` entries each (a multiple of 32, at least 32
// words' worth past K + 31), copy p entry j = box offset of local cell j - p
// or T.dummy.
hipError_t launch_pack_bits(const uint8_t *bytes, uint32_t *words, uint64_t cells, int grid, hipStream_t st);
hipError_t launch_unpack_bits(const uint32_t *words, uint8_t *bytes, uint64_t cells, int grid, hipStream_t st);
uint32_t packed_stage_words(const TileParams &T);
bool packed_fits(const TileParams &T);
hipError_t launch_step_packed(const TileParams &T, const uint16_t *lutw, uint32_t stride, const uint32_t *in,
                              uint32_t *out, uint32_t rule, int cu_count, hipStream_t st);

}  // namespace nbb
