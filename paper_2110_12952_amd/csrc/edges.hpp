// The tiled compact step in edge-record form (k_step_edges) and its launchers.
// Included by edges_inst.hip, which is compiled once per (BATCH, RULE) so the
// instantiations build in parallel.
//
// Section 3's stencil procedure on the blocked approach, for compact storage:
// tile t = compact cells [t K, (t+1) K) is one level-m copy of the fractal,
// cut into level-q blocks whose CB cells are consecutive in compact order and
// fill the same positions of a BS x BS square in every block.  Per tile a
// work-group of 256 threads
//   1. loads each block's CB bytes into registers (one load per block; every
//      thread keeps its blocks for the whole launch), unpacks them into BS row
//      dwords with v_perm (byte c of row r = cell (c, r), 0 off the fractal)
//      and writes the block's edges (top row, bottom row, left column, right
//      column) as its record in four LDS dword arrays, records in block order
//      so that a wavefront's lanes write consecutive dwords; the blocks of
//      the eight neighbour tiles that touch the tile's blocks (halo items)
//      write records after them (zeros where a neighbour tile does not
//      exist);
//   2. reads, per block, the bottom rows of the three records above, the top
//      rows of the three below and the facing columns of the two beside it
//      (numbers from the plan; a record of zeros where there is no block):
//      with the block's own rows these are its whole (BS+2)-square window.
//      Row 3-sums four positions per dword (SWAR: bytes never exceed 9),
//      the rule per byte, v_perm back into compact order, and the block's CB
//      next states go straight to global memory.
// Work-groups are persistent over XCD-contiguous tile ranges; the next
// tile's loads are issued before the current tile's rule, and its neighbour
// tiles travel through LDS two tiles ahead.
//
// BATCH: tiles of many instances of one plan in an arena, as in the
// byte-scatter form (k_step_tiled): batch tile g is local tile rec[2g+1]
// (low 31 bits) of the state at byte 16 rec[2g] of the arena.
//
// RULE: 0 = B3/S23 (born with 3, survives with 2 or 3 <=> (neighbours |
// self) == 3), 1 = any rule without birth or survival at 8 (two v_perm table
// look-ups), 2 = any rule (per-byte bit extract from the rule word).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "device_common.hpp"

namespace nbb {

template <int NSRC>
struct RawBlock {
    uint32_t d[NSRC];
};

// 4 NSRC bytes from any byte address (gfx950 global loads need no alignment).
template <int NSRC>
__device__ __forceinline__ RawBlock<NSRC> load_block(const uint8_t *p) {
    RawBlock<NSRC> r;
    __builtin_memcpy(&r, p, 4 * NSRC);
    return r;
}

// The block's bytes were loaded ending at its last cell: move them down by
// sh bytes (0 < sh < 4 NSRC, uniform).
template <int NSRC>
__device__ __forceinline__ void shift_block(RawBlock<NSRC> &r, uint32_t sh) {
    uint32_t d[NSRC + 1];
#pragma unroll
    for (int i = 0; i < NSRC; ++i) d[i] = r.d[i];
    d[NSRC] = 0;
    for (uint32_t w = 0; w < (sh >> 2); ++w) {
#pragma unroll
        for (int i = 0; i < NSRC; ++i) d[i] = d[i + 1];
    }
#pragma unroll
    for (int i = 0; i < NSRC; ++i) r.d[i] = alignbyte(d[i + 1], d[i], sh & 3);
}

// SEL: which of the plan's v_perm selectors pick any byte (bit r: unpack01[r],
// 4 + r: unpack23[r], 8 + d: pack01[d], 12 + d: pack23[d]); a form compiled
// for a plan's mask leaves out the permutes whose selectors pick nothing.
// kAllSel: every selector may pick bytes (the general form).
constexpr uint32_t kAllSel = 0xFFFFu;
constexpr uint32_t kNoBytes = 0x0C0C0C0Cu;  // a selector picking no byte (12: zero)
inline uint32_t edge_sel_mask(const EdgeParams &E) {
    uint32_t m = 0;
    for (int i = 0; i < 4; ++i) {
        m |= uint32_t(E.unpack01[i] != kNoBytes) << i;
        m |= uint32_t(E.unpack23[i] != kNoBytes) << (4 + i);
        m |= uint32_t(E.pack01[i] != kNoBytes) << (8 + i);
        m |= uint32_t(E.pack23[i] != kNoBytes) << (12 + i);
    }
    return m;
}

template <int BS, int NSRC, uint32_t SEL>
__device__ __forceinline__ void unpack_rows(const EdgeParams &E, const RawBlock<NSRC> &r, uint32_t (&row)[BS]) {
#pragma unroll
    for (int rr = 0; rr < BS; ++rr) {
        uint32_t v = 0;
        if (SEL & (1u << rr)) v = __builtin_amdgcn_perm(r.d[1], r.d[0], E.unpack01[rr]);
        if (NSRC == 4 && (SEL & (16u << rr))) v |= __builtin_amdgcn_perm(r.d[3], r.d[2], E.unpack23[rr]);
        row[rr] = v;
    }
}

// v_perm selector: bytes s0..s3 (s0 the lowest); 0-3 pick the second
// operand's bytes, 4-7 the first's, 12 a zero byte.
constexpr uint32_t sel4(uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3) {
    return s0 | (s1 << 8) | (s2 << 16) | (s3 << 24);
}

// The block's record: top row, bottom row, left column, right column (byte r
// of a column = row r).
template <int BS>
__device__ __forceinline__ uint4 edge_record(const uint32_t (&row)[BS]) {
    uint32_t left, right;
    if (BS == 4) {
        const uint32_t l01 = __builtin_amdgcn_perm(row[1], row[0], sel4(0, 4, 12, 12));
        const uint32_t l23 = __builtin_amdgcn_perm(row[BS - 1], row[2], sel4(0, 4, 12, 12));
        left = __builtin_amdgcn_perm(l23, l01, sel4(0, 1, 4, 5));
        const uint32_t r01 = __builtin_amdgcn_perm(row[1], row[0], sel4(3, 7, 12, 12));
        const uint32_t r23 = __builtin_amdgcn_perm(row[BS - 1], row[2], sel4(3, 7, 12, 12));
        right = __builtin_amdgcn_perm(r23, r01, sel4(0, 1, 4, 5));
    } else {
        const uint32_t l01 = __builtin_amdgcn_perm(row[1], row[0], sel4(0, 4, 12, 12));
        left = __builtin_amdgcn_perm(row[BS - 1], l01, sel4(0, 1, 4, 12));
        const uint32_t r01 = __builtin_amdgcn_perm(row[1], row[0], sel4(2, 6, 12, 12));
        right = __builtin_amdgcn_perm(row[BS - 1], r01, sel4(0, 1, 6, 12));
    }
    return make_uint4(row[0], row[BS - 1], left, right);
}

// Stores the CB compact bytes of w (any alignment).  CB is uniform, so the
// choice below is scalar branches only (none when CB is known at compile
// time: CBC, 0 if not).
template <int CBC>
__device__ __forceinline__ void store_cells(const uint32_t (&w)[4], uint32_t CB_, uint8_t *p) {
    const uint32_t CB = CBC ? uint32_t(CBC) : CB_;
    if (CB == 16) {
        store_u64(p, w[0], w[1]);
        store_u64(p + 8, w[2], w[3]);
    } else if (CB > 8) {
        store_u64(p, w[0], w[1]);
        uint32_t r = CB - 8, x = w[2];
        p += 8;
        if (r >= 4) {
            store_u32(p, x);
            p += 4;
            r -= 4;
            x = w[3];
        }
        if (r >= 2) {
            store_u16(p, x);
            p += 2;
            r -= 2;
            x >>= 16;
        }
        if (r) store_u8(p, x);
    } else if (CB == 8) {
        store_u64(p, w[0], w[1]);
    } else if (CB > 4) {
        store_u32(p, w[0]);
        store_u32(p + (CB - 4), alignbyte(w[1], w[0], CB - 4));
    } else if (CB == 4) {
        store_u32(p, w[0]);
    } else if (CB >= 2) {
        store_u16(p, w[0]);
        if (CB == 3) store_u16(p + 1, w[0] >> 8);
    } else {
        store_u8(p, w[0]);
    }
}

// The records in LDS: four dword arrays (top rows, bottom rows, left
// columns, right columns) of SR entries each; a record is addressed by 4 x
// its number, the array by an instruction offset.
template <uint32_t SR>
struct EdgeRecs {
    uint8_t *lds;
    __device__ __forceinline__ uint32_t &at(uint32_t k, uint32_t a4) const {
        return *reinterpret_cast<uint32_t *>(lds + a4 + k * SR * 4);
    }
    __device__ __forceinline__ void put(uint32_t a4, const uint4 &r) const {
        at(0, a4) = r.x;
        at(1, a4) = r.y;
        at(2, a4) = r.z;
        at(3, a4) = r.w;
    }
};
constexpr uint32_t kTop = 0, kBot = 1, kLeft = 2, kRight = 3;

// A block's eight neighbouring records (4 x their numbers).
struct EdgeNbrs {
    uint32_t L, R, A, B, AL, AR, BL, BR;
};

// Next states of one block, rows in next[0..BS) (byte c = column c).
template <int BS, bool EDGE, int RULE, uint32_t SR>
__device__ __forceinline__ void edge_block_rule(const EdgeRecs<SR> &g, const EdgeNbrs &nb, const uint32_t (&o)[BS],
                                                uint32_t rule, const RuleTables &RT, uint32_t (&next)[4]) {
    // the facing columns of the left and right neighbours
    const uint32_t Lc = g.at(kRight, nb.L), Rc = g.at(kLeft, nb.R);
    // centre rows above and below (bottom row of the record above, top row of the one below)
    const uint32_t aC = g.at(kBot, nb.A), bC = g.at(kTop, nb.B);
    // lo: byte c = position c - 1, hi: byte c = position c + 1, for each window row
    uint32_t lo[BS], hi[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) {
        lo[r] = __builtin_amdgcn_perm(o[r], Lc, sel4(r, 4, 5, 6));
        hi[r] = BS == 4 ? __builtin_amdgcn_perm(Rc, o[r], sel4(1, 2, 3, 4 + r))
                        : __builtin_amdgcn_perm(Rc, o[r], sel4(1, 2, 4 + r, 12));
    }
    uint32_t n[BS];
    if (EDGE) {
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            const uint32_t up = r == 0 ? aC : o[r - 1], dn = r == BS - 1 ? bC : o[r + 1];
            n[r] = up + dn + lo[r] + hi[r];
        }
    } else {
        const uint32_t aL = g.at(kBot, nb.AL), aR = g.at(kBot, nb.AR);
        const uint32_t bL = g.at(kTop, nb.BL), bR = g.at(kTop, nb.BR);
        uint32_t H[BS + 2];
        if (BS == 4) {
            H[0] = alignbyte(aC, aL, 3) + aC + alignbyte(aR, aC, 1);
            H[BS + 1] = alignbyte(bC, bL, 3) + bC + alignbyte(bR, bC, 1);
        } else {
            H[0] = __builtin_amdgcn_perm(aC, aL, sel4(2, 4, 5, 6)) + aC +
                   __builtin_amdgcn_perm(aR, aC, sel4(1, 2, 4, 12));
            H[BS + 1] = __builtin_amdgcn_perm(bC, bL, sel4(2, 4, 5, 6)) + bC +
                        __builtin_amdgcn_perm(bR, bC, sel4(1, 2, 4, 12));
        }
#pragma unroll
        for (int r = 0; r < BS; ++r) H[r + 1] = lo[r] + o[r] + hi[r];
#pragma unroll
        for (int r = 0; r < BS; ++r) n[r] = H[r] + H[r + 1] + H[r + 2] - o[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r >= BS) {
            next[r] = 0;
            continue;
        }
        if (RULE == 0) {
            next[r] = __builtin_amdgcn_perm(0u, 0x01000000u, n[r] | o[r]);
        } else if (RULE == 1) {
            const uint32_t born = __builtin_amdgcn_perm(RT.born_hi, RT.born_lo, n[r]);
            const uint32_t surv = __builtin_amdgcn_perm(RT.surv_hi, RT.surv_lo, n[r]);
            const uint32_t smask = __builtin_amdgcn_perm(0u, 0x0000FF00u, o[r]);  // 0xFF where alive
            next[r] = (surv & smask) | (born & ~smask);
        } else {
            // v_bfe takes its offset from the low 5 bits of the operand
            const uint32_t I = n[r] + (o[r] << 4);
            uint32_t v = __builtin_amdgcn_ubfe(rule, I, 1);
#pragma unroll
            for (int c = 1; c < BS; ++c) v |= __builtin_amdgcn_ubfe(rule, I >> (8 * c), 1) << (8 * c);
            next[r] = v;
        }
    }
}

template <int BS, int NSRC, int BPT, int HPT, bool BATCH, bool EDGE, int RULE, int CBC, uint32_t SEL>
__global__ __launch_bounds__(256) void k_step_edges(EdgeParams E, const uint8_t *__restrict__ in,
                                                    uint8_t *__restrict__ out, uint32_t rule,
                                                    const uint32_t *__restrict__ rec) {
    extern __shared__ __align__(16) uint8_t lds_e[];
    constexpr uint32_t kLanes = BATCH ? 10 : 8;  // neighbour tiles (+ record) per tile
    constexpr uint32_t kLane0 = 256 - kLanes;
    __shared__ uint32_t nbr[2][kLanes];
    const uint32_t tid = threadIdx.x;
    const uint32_t K = E.K, CB = E.CB;
    const XcdRange R = xcd_range(blockIdx.x, gridDim.x, E.ntiles);
    auto entry = [&](uint64_t t, uint32_t l) -> uint32_t {
        return (!BATCH || l < 8) ? E.nbr[t * 8 + l] : rec[t * 2 + (l - 8)];
    };

    constexpr uint32_t SR = edge_rec_stride(BPT, HPT);
    for (uint32_t o = tid * 16; o < 16 * SR; o += 256 * 16)
        *reinterpret_cast<uint4 *>(lds_e + o) = make_uint4(0, 0, 0, 0);
    const RuleTables RT = rule_tables(rule);
    // this thread's blocks and halo items (the same in every tile)
    EdgeNbrs nb[BPT];
    uint32_t own[BPT], boff[BPT], loff[BPT];
    bool bnear[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const uint32_t bi = min(tid + 256 * j, E.nblk - 1);
        const uint4 w = *reinterpret_cast<const uint4 *>(E.blk + 4 * bi);
        nb[j] = EdgeNbrs{(w.x & 0xFFFFu) * 4, (w.x >> 16) * 4, (w.y & 0xFFFFu) * 4, (w.y >> 16) * 4,
                         (w.z & 0xFFFFu) * 4, (w.z >> 16) * 4, (w.w & 0xFFFFu) * 4, (w.w >> 16) * 4};
        own[j] = bi * 4;
        boff[j] = bi * CB;
        bnear[j] = boff[j] + 4 * NSRC > K;
        loff[j] = boff[j] - (bnear[j] ? E.nsh : 0u);
    }
    uint32_t hdir[HPT], hoff[HPT], hrec[HPT];
    bool hnear[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const uint32_t h = tid + 256 * j;
        const bool ok = h < E.nhalo;
        const uint32_t w0 = ok ? E.halo[2 * h] : 0u, w1 = ok ? E.halo[2 * h + 1] : 0u;
        hdir[j] = ok ? (w0 >> 29) : 8u;  // 8: no item
        hnear[j] = (w1 >> 31) != 0;
        hoff[j] = (w0 & 0x1FFFFFFFu) * CB - (hnear[j] ? E.nsh : 0u);
        hrec[j] = (w1 & 0xFFFFu) * 4;
    }
    if (tid >= kLane0) {
        if (R.first < R.end) nbr[0][tid - kLane0] = entry(R.first, tid - kLane0);
        if (R.first + R.step < R.end) nbr[1][tid - kLane0] = entry(R.first + R.step, tid - kLane0);
    }
    __syncthreads();

    // where a tile lives: its state array and local index
    const uint8_t *src = in;
    uint8_t *dst = out;
    uint32_t local = 0;
    auto locate = [&](uint64_t t, const uint32_t *e) {
        if (BATCH) {
            const uint64_t base = uint64_t(__builtin_amdgcn_readfirstlane(e[8])) << 4;
            src = in + base;
            dst = out + base;
            local = __builtin_amdgcn_readfirstlane(e[9]) & 0x7FFFFFFFu;
        } else {
            local = uint32_t(t);
        }
    };
    RawBlock<NSRC> raw[BPT], hraw[HPT];
    auto prefetch = [&](const uint32_t *e) {
        const uint8_t *tb = src + uint64_t(local) * K;
#pragma unroll
        for (int j = 0; j < BPT; ++j)
            if (tid + 256 * j < E.nblk) raw[j] = load_block<NSRC>(tb + loff[j]);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const uint32_t nt = hdir[j] < 8 ? e[hdir[j]] : kOutside;
            if (nt != kOutside) {
                hraw[j] = load_block<NSRC>(src + uint64_t(nt) * K + hoff[j]);
            } else {
#pragma unroll
                for (int i = 0; i < NSRC; ++i) hraw[j].d[i] = 0;
            }
        }
    };
    if (R.first < R.end) {
        locate(R.first, nbr[0]);
        prefetch(nbr[0]);
    }

    const EdgeRecs<SR> grid{lds_e};
    uint32_t it = 0;
    for (uint64_t t64 = R.first; t64 < R.end; t64 += R.step, ++it) {
        uint8_t *gout = dst + uint64_t(local) * K;
        // 1. records of the tile's blocks (kept as rows) and of the halo blocks
        uint32_t rows[BPT][BS];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            if (tid + 256 * j < E.nblk) {
                if (bnear[j]) shift_block<NSRC>(raw[j], E.nsh);
                unpack_rows<BS, NSRC, SEL>(E, raw[j], rows[j]);
                grid.put(own[j], edge_record<BS>(rows[j]));
            }
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hdir[j] < 8) {
                if (hnear[j]) shift_block<NSRC>(hraw[j], E.nsh);
                uint32_t hr[BS];
                unpack_rows<BS, NSRC, SEL>(E, hraw[j], hr);
                grid.put(hrec[j], edge_record<BS>(hr));
            }
        }
        __syncthreads();
        // 2. loads of the next tile
        if (t64 + R.step < R.end) {
            const uint32_t *e = nbr[(it + 1) & 1];
            locate(t64 + R.step, e);
            prefetch(e);
        }
        uint32_t nb2 = kOutside;
        if (tid >= kLane0 && t64 + 2 * R.step < R.end) nb2 = entry(t64 + 2 * R.step, tid - kLane0);
        // 3. the rule per block, next states straight to global memory
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            if (tid + 256 * j < E.nblk) {
                uint32_t next[4];
                edge_block_rule<BS, EDGE, RULE, SR>(grid, nb[j], rows[j], rule, RT, next);
                uint32_t w[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    uint32_t v = 0;
                    if (SEL & (256u << d)) v = __builtin_amdgcn_perm(next[1], next[0], E.pack01[d]);
                    if (BS >= 3 && (SEL & (4096u << d))) v |= __builtin_amdgcn_perm(next[3], next[2], E.pack23[d]);
                    w[d] = v;
                }
                store_cells<CBC>(w, CB, gout + boff[j]);
            }
        }
        // the records are read until here; the next tile's come after
        __syncthreads();
        if (tid >= kLane0) nbr[it & 1][tid - kLane0] = nb2;
    }
}

// Persistent launch: as many work-groups as can be resident at once, capped
// by the tiles.
template <int BS, int NSRC, int BPT, int HPT, bool BATCH, bool EDGE, int RULE, int CBC, uint32_t SEL>
static hipError_t launch_edges_t(const EdgeParams &E, const uint8_t *in, uint8_t *out, uint32_t rule,
                                 const uint32_t *rec, int cu_count, EdgeCaps caps, hipStream_t st) {
    const size_t lds = edge_lds_bytes(BPT, HPT);
    static std::atomic<uint64_t> cached{0};  // lds << 32 | per_cu
    int per_cu = 0;
    const uint64_t c = cached.load(std::memory_order_relaxed);
    if (c >> 32 == lds && (c & 0xFFFFFFFFu)) {
        per_cu = int(c & 0xFFFFFFFFu);
    } else {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_step_edges<BS, NSRC, BPT, HPT, BATCH, EDGE, RULE, CBC, SEL>, 256, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        cached.store(uint64_t(lds) << 32 | uint32_t(per_cu), std::memory_order_relaxed);
    }
    const int cap = BPT == 1 ? caps.one : caps.more;
    if (cap > 0) per_cu = std::min(per_cu, cap);
    const uint64_t grid = std::min<uint64_t>(uint64_t(per_cu) * cu_count, E.ntiles);
    if (!grid) return hipSuccess;
    hipLaunchKernelGGL((k_step_edges<BS, NSRC, BPT, HPT, BATCH, EDGE, RULE, CBC, SEL>), dim3(uint32_t(grid)), dim3(256), lds,
                       st, E, in, out, rule, rec);
    return hipGetLastError();
}
template <int BS, int NSRC, bool BATCH, bool EDGE, int RULE, int CBC = 0, uint32_t SEL = kAllSel>
static hipError_t launch_edges_s(const EdgeParams &E, const uint8_t *in, uint8_t *out, uint32_t rule,
                                 const uint32_t *rec, int cu_count, EdgeCaps caps, hipStream_t st) {
    uint32_t bpt = 0, hpt = 0;
    if (!edge_case(E.nblk, E.nhalo, &bpt, &hpt)) return hipErrorInvalidValue;
#define NBB_EDGES_CASE(B, H)                                                                              \
    if (bpt == B && hpt == H)                                                                             \
    return launch_edges_t<BS, NSRC, B, H, BATCH, EDGE, RULE, CBC, SEL>(E, in, out, rule, rec, cu_count, caps, st)
    NBB_EDGES_CASE(1, 1);
    NBB_EDGES_CASE(2, 1);
    NBB_EDGES_CASE(4, 1);
    NBB_EDGES_CASE(1, 2);
    NBB_EDGES_CASE(2, 2);
    NBB_EDGES_CASE(4, 2);
#undef NBB_EDGES_CASE
    return hipErrorInvalidValue;
}
// Forms compiled for particular plans: (block side, source dwords, cells per
// block, selector mask).  The triangle F^{3,2} with offsets (0,0), (1,0),
// (0,1) at block level 2 needs 4 of the 8 unpacking and 5 of the 12 packing
// permutes and stores 8 + 1 bytes per block: 25.0 us per generation at r16
// against 26.3 in the general form.  (Compiled the same way for the carpet
// at level 1 it ran 62.7 us against 61.5, so the carpet, H and chandelier
// plans keep the general form.)  Any other plan takes the general form.
struct EdgeSpec {
    uint32_t BS, nsrc, CB, sel;
};
constexpr EdgeSpec kSpecTriangle{4, 4, 9, 0x6387u};

// shape: BS 3 or 4, and 2 or 4 source dwords per block
template <bool BATCH, bool EDGE, int RULE>
static hipError_t launch_edges_shape(const EdgeParams &E, uint32_t BS, uint32_t nsrc, const uint8_t *in,
                                     uint8_t *out, uint32_t rule, const uint32_t *rec, int cu_count, EdgeCaps caps,
                                     hipStream_t st) {
    const uint32_t sel = edge_sel_mask(E);
    auto is = [&](const EdgeSpec &p) { return BS == p.BS && nsrc == p.nsrc && E.CB == p.CB && sel == p.sel; };
#define NBB_EDGES_SPEC(P)                                                                                        \
    if (is(P))                                                                                                   \
    return launch_edges_s<P.BS, P.nsrc, BATCH, EDGE, RULE, P.CB, P.sel>(E, in, out, rule, rec, cu_count,         \
                                                                        caps, st)
    NBB_EDGES_SPEC(kSpecTriangle);
#undef NBB_EDGES_SPEC
    if (BS == 3 && nsrc == 2)
        return launch_edges_s<3, 2, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    if (BS == 3 && nsrc == 4)
        return launch_edges_s<3, 4, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    if (BS == 4 && nsrc == 4)
        return launch_edges_s<4, 4, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    return hipErrorInvalidValue;
}

}  // namespace nbb
