// The tiled compact step (k_step_tiled) and its launchers.  Included by
// tiled_inst.hip, which is compiled once per (BATCH, TEAM, EDGE) so that the
// many instantiations build in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "device_common.hpp"

namespace nbb {

#ifndef NBB_TILED_WAVES_PER_SIMD
#define NBB_TILED_WAVES_PER_SIMD 1
#endif
// Most resident work-groups per CU of the persistent launch.
#ifndef NBB_TILED_MAX_PER_CU
#define NBB_TILED_MAX_PER_CU 7
#endif
// Compact step, tiled (section 3, blocked approach, applied to compact
// storage).  Tile t = compact cells [t K, (t+1) K), K = k^m: one level-m copy
// of the fractal, covering the S x S block (S = s^m) of the box whose corner
// is S * lambda_{r-m}(t).  Since every tile is the same copy of F_m, the
// position of local cell i inside its block (lut0) and the list of neighbour
// cells that touch the block (halo) are the same for every tile; only the
// eight neighbour tiles differ.  Per tile a work-group
//   1. scatters the tile's K bytes and its halo into an LDS box of
//      rows x W bytes (cells outside the fractal stay 0),
//   2. evaluates the rule for each block of CB cells (block_rows: four
//      positions per dword), gathers the block's member bytes into compact
//      order (block_store: v_perm) and stores its CB next states, which are
//      consecutive compact cells, straight to global memory.
// Work-groups are persistent and walk an XCD-contiguous range of tiles as a
// software pipeline: the next tile's bytes and halo are loaded into registers
// while the current tile computes, and the neighbour tiles are found two
// tiles ahead by a few threads and passed on through LDS.
//
// BATCH: the tiles of many independent fractals that share the tile plan
// (same k, s, offsets and m, any r), each state at its own place in one
// arena.  Batch tile g is local tile rec[2g+1] (bit 31: the tail flag of
// tile_prefetch) of the state at byte 16 rec[2g] of the arena, and T.nbr
// holds its eight neighbours as local tiles of the same state.  The record
// travels through LDS with the neighbour tiles, two tiles ahead.
//
// TEAM: threads per tile.  256 = the whole work-group works on one tile at a
// time.  64 = each wavefront is a worker of its own with its own LDS box and
// its own range of tiles, synchronising only within the wavefront; for small
// tiles, whose few chunks, halo cells and blocks leave most of a work-group
// idle, four independent pipelines per work-group hide more memory latency.
template <int TEAM>
__device__ __forceinline__ void team_sync() {
    if (TEAM == 256) {
        __syncthreads();
    } else {
        // one wavefront: its LDS accesses complete in program order, so only
        // the compiler must be kept from moving them across this point
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int BS, int CPT, int HPT, int BPT, bool BATCH, int TEAM, bool EDGE, int ROWS>
__global__ __launch_bounds__(256, NBB_TILED_WAVES_PER_SIMD) void k_step_tiled(
    MapParams P, TileParams T, const uint8_t *__restrict__ in, uint8_t *__restrict__ out, uint32_t rule,
    const uint32_t *__restrict__ rec) {
    extern __shared__ __align__(16) uint8_t lds_all[];
    constexpr uint32_t kTeams = 256 / TEAM;
    constexpr uint32_t kLanes = BATCH ? 10 : 8;  // neighbour tiles (+ record) per tile
    constexpr uint32_t kLane0 = TEAM - kLanes;
    __shared__ uint32_t nbr_all[kTeams][2][kLanes];
    // the team index is uniform across a wavefront: keep it (and every tile
    // index derived from it) in scalar registers
    const uint32_t team = TEAM == 256 ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x / TEAM);
    const uint32_t tid = TEAM == 256 ? threadIdx.x : threadIdx.x % TEAM;
    uint8_t *lds = lds_all + team * T.lds_total;
    uint8_t *box = lds;
    uint32_t (*nbr)[kLanes] = nbr_all[team];
    const uint32_t K = T.K;
    const XcdRange R = xcd_range(blockIdx.x, gridDim.x, T.ntiles, team, kTeams);
    // word l of the per-tile LDS entry of tile t
    auto entry = [&](uint64_t t, uint32_t l) -> uint32_t {
        return (!BATCH || l < 8) ? T.nbr[t * 8 + l] : rec[t * 2 + (l - 8)];
    };

    for (uint32_t o = threadIdx.x * 16; o < kTeams * T.lds_total; o += 256 * 16)
        *reinterpret_cast<uint4 *>(lds_all + o) = make_uint4(0, 0, 0, 0);
    const RuleTables RT = rule_tables(rule);
    uint32_t hsrc[HPT], hdst[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const uint32_t h = tid + TEAM * j;
        const bool ok = h < T.halo_count;
        hsrc[j] = ok ? T.halo_src[h] : kOutside;
        hdst[j] = ok ? T.halo_dst[h] : T.dummy;
    }
    // Block window corners (the same for every tile).
    uint32_t blk[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) blk[j] = T.lut1[min(tid + TEAM * j, T.nblk - 1)];
    // Neighbour tiles go through LDS two tiles ahead: the last kLanes threads
    // of the team load the entries of tile it+2 after the first barrier of
    // tile it and publish them after its second barrier.
    if (tid >= kLane0) {
        if (R.first < R.end) nbr[0][tid - kLane0] = entry(R.first, tid - kLane0);
        if (R.first + R.step < R.end) nbr[1][tid - kLane0] = entry(R.first + R.step, tid - kLane0);
    }
    __syncthreads();

    // Where tile t lives: its state array, local index and tail flag.
    const uint8_t *src = in;
    uint8_t *dst = out;
    uint32_t local = 0, cells = T.cells;
    bool tail = false;
    auto locate = [&](uint64_t t, const uint32_t *e) {
        if (BATCH) {
            const uint64_t base = uint64_t(__builtin_amdgcn_readfirstlane(e[8])) << 4;
            const uint32_t w = __builtin_amdgcn_readfirstlane(e[9]);
            src = in + base;
            dst = out + base;
            local = w & 0x7FFFFFFFu;
            tail = (w >> 31) != 0;
            cells = (local + 1) * K;  // only read when tail is set: the tile is the last one
        } else {
            local = uint32_t(t);
            tail = (local * K + K == T.cells) && (T.cells & 15);
        }
    };

    TilePrefetch<CPT, HPT> pf;
    uint32_t pf_ph = 0xFFFFFFFFu;  // no offsets loaded yet
    if (R.first < R.end) {
        locate(R.first, nbr[0]);
        tile_prefetch<TEAM, CPT, HPT, !BATCH>(T, src, local, tail, cells, nbr[0], hsrc, pf, pf_ph);
    }

    const uint32_t *box32 = reinterpret_cast<const uint32_t *>(box);
    const uint32_t W4 = T.W >> 2;
    uint32_t it = 0;
    for (uint64_t t64 = R.first; t64 < R.end; t64 += R.step, ++it) {
        const uint32_t B = local * K;  // first cell of the tile in its state array (< 2^32)
        uint8_t *gout = dst + B;
        const uint32_t ph = B & 15;
        const uint32_t nchunks = (ph + K + 15) >> 4;
        // 1. scatter the prefetched tile and halo into the box.  Offsets of
        //    bytes outside the tile point at a never-read byte.
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (tid + TEAM * j < nchunks) {
                const uint32_t v[4] = {pf.v[j].x, pf.v[j].y, pf.v[j].z, pf.v[j].w};
                const uint32_t e[8] = {pf.e[j][0].x, pf.e[j][0].y, pf.e[j][0].z, pf.e[j][0].w,
                                       pf.e[j][1].x, pf.e[j][1].y, pf.e[j][1].z, pf.e[j][1].w};
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    box[(e[b >> 1] >> (16 * (b & 1))) & 0xFFFFu] = uint8_t(v[b >> 2] >> (8 * (b & 3)));
            }
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) box[hdst[j]] = uint8_t(pf.halo[j]);
        team_sync<TEAM>();

        // 2. start loading the next tile
        if (t64 + R.step < R.end) {
            const uint32_t *e = nbr[(it + 1) & 1];
            locate(t64 + R.step, e);
            tile_prefetch<TEAM, CPT, HPT, !BATCH>(T, src, local, tail, cells, e, hsrc, pf, pf_ph);
        }
        uint32_t nb2 = kOutside;
        if (tid >= kLane0 && t64 + 2 * R.step < R.end) nb2 = entry(t64 + 2 * R.step, tid - kLane0);

        // 3. rule per block, next states straight to global memory (block b
        //    holds the tile's cells [b CB, (b+1) CB))
        if (rule == kRuleB3S23) {
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const uint32_t bi = tid + TEAM * j;
                if (bi < T.nblk) {  // waves with no block left skip the work
                    uint32_t next[4];
                    block_rows<BS, 0, false, ROWS>(box32, W4, blk[j], rule, RT, next);
                    block_store<BS>(T, next, gout + bi * T.CB);
                }
            }
        } else if (RT.perm) {
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const uint32_t bi = tid + TEAM * j;
                if (bi < T.nblk) {
                    uint32_t next[4];
                    block_rows<BS, 1, EDGE, ROWS>(box32, W4, blk[j], rule, RT, next);
                    block_store<BS>(T, next, gout + bi * T.CB);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const uint32_t bi = tid + TEAM * j;
                if (bi < T.nblk) {
                    uint32_t next[4];
                    block_rows<BS, 2, EDGE, ROWS>(box32, W4, blk[j], rule, RT, next);
                    block_store<BS>(T, next, gout + bi * T.CB);
                }
            }
        }
        // the box is read until here; the next tile's scatter comes after
        team_sync<TEAM>();
        if (tid >= kLane0) nbr[it & 1][tid - kLane0] = nb2;
    }
}

// Persistent launch: as many work-groups as can be resident at once (the
// occupancy of this instantiation for its LDS size), capped by the tiles.
template <int BS, int CPT, int HPT, int BPT, bool BATCH, int TEAM, bool EDGE, int ROWS>
static hipError_t launch_tiled_t(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                                 uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    constexpr uint32_t kTeams = 256 / TEAM;
    const size_t lds = size_t(kTeams) * T.lds_total;
    // resident work-groups per CU for this instantiation and LDS size; the
    // last answer is kept (one query per plan, not per launch)
    static std::atomic<uint64_t> cached{0};  // lds << 32 | per_cu
    int per_cu = 0;
    const uint64_t c = cached.load(std::memory_order_relaxed);
    if (c >> 32 == lds && (c & 0xFFFFFFFFu)) {
        per_cu = int(c & 0xFFFFFFFFu);
    } else {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_step_tiled<BS, CPT, HPT, BPT, BATCH, TEAM, EDGE, ROWS>, 256, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        cached.store(uint64_t(lds) << 32 | uint32_t(per_cu), std::memory_order_relaxed);
    }
    // More than seven work-groups per CU measured slower where the occupancy
    // allows eight (H r10: 186 us per generation at 8, 166 us at 7; the
    // batch's H group 124 -> 111 us); at 7 and below nothing changes.
    constexpr int kMaxPerCU = NBB_TILED_MAX_PER_CU;
    const uint64_t grid = std::min<uint64_t>(uint64_t(std::min(per_cu, kMaxPerCU)) * cu_count,
                                             (T.ntiles + kTeams - 1) / kTeams);
    hipLaunchKernelGGL((k_step_tiled<BS, CPT, HPT, BPT, BATCH, TEAM, EDGE, ROWS>), dim3(uint32_t(grid)), dim3(256), lds, st,
                       P, T, in, out, rule, rec);
    return hipGetLastError();
}
template <int BS, int CPT, int HPT, bool BATCH, int TEAM, bool EDGE, int ROWS>
static hipError_t launch_tiled_b(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                                 uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    const uint32_t bpt = (T.nblk + TEAM - 1) / TEAM;
    if (bpt <= 1) return launch_tiled_t<BS, CPT, HPT, 1, BATCH, TEAM, EDGE, ROWS>(P, T, in, out, rule, rec, cu_count, st);
    if (bpt <= 2) return launch_tiled_t<BS, CPT, HPT, 2, BATCH, TEAM, EDGE, ROWS>(P, T, in, out, rule, rec, cu_count, st);
    if (bpt <= 4) return launch_tiled_t<BS, CPT, HPT, 4, BATCH, TEAM, EDGE, ROWS>(P, T, in, out, rule, rec, cu_count, st);
    return hipErrorInvalidValue;
}
template <int BS, bool BATCH, int TEAM, bool EDGE, int ROWS>
static hipError_t launch_tiled_s(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                                 uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    const uint32_t cpt = (T.K + 30 + 16 * TEAM - 1) / (16 * TEAM);
    const uint32_t hpt = (T.halo_count + TEAM - 1) / TEAM;
#define NBB_TILED_CASE(C, H) \
    if (cpt <= C && hpt <= H) return launch_tiled_b<BS, C, H, BATCH, TEAM, EDGE, ROWS>(P, T, in, out, rule, rec, cu_count, st)
    NBB_TILED_CASE(1, 1);
    NBB_TILED_CASE(1, 2);
    NBB_TILED_CASE(1, 4);
    NBB_TILED_CASE(2, 1);
    NBB_TILED_CASE(2, 2);
    NBB_TILED_CASE(2, 4);
#undef NBB_TILED_CASE
    return hipErrorInvalidValue;
}
template <bool BATCH, int TEAM, bool EDGE>
static hipError_t launch_tiled_bs(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                                  uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    switch (T.BS) {
        case 2: return launch_tiled_s<2, BATCH, TEAM, EDGE, 2>(P, T, in, out, rule, rec, cu_count, st);
        case 3:  // 3x3 blocks whose third row holds no cell get the two-row form
            return T.brows == 2 ? launch_tiled_s<3, BATCH, TEAM, EDGE, 2>(P, T, in, out, rule, rec, cu_count, st)
                                : launch_tiled_s<3, BATCH, TEAM, EDGE, 3>(P, T, in, out, rule, rec, cu_count, st);
        case 4: return launch_tiled_s<4, BATCH, TEAM, EDGE, 4>(P, T, in, out, rule, rec, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace nbb
