// The tiled compact step in edge-record form (k_step_edges) and its launchers.
// Included by edges_inst.hip, which is compiled once per (BATCH, RULE) so the
// instantiations build in parallel.
//
// Section 3's stencil procedure on the blocked approach, for compact storage:
// tile t = compact cells [t K, (t+1) K) is one level-m copy of the fractal,
// cut into level-q blocks whose CB cells are consecutive in compact order and
// fill the same positions of a BS x BS square in every block.  Per tile a
// work-group of 256 threads
//   1. loads each block's CB bytes into registers (one load of an 8-byte
//      aligned window per block, moved into place with v_alignbyte; every
//      thread keeps its blocks for the whole launch), unpacks them into BS
//      row dwords with v_perm (byte c of row r = cell (c, r), 0 off the fractal)
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
// Work-groups are persistent over XCD-contiguous tile ranges.  A tile's
// loads are issued two tiles ahead of its rule (two register sets, the loop
// unrolled twice so that each has fixed registers) and its neighbour tiles'
// numbers four tiles ahead (through registers, then LDS); no load, store or
// use of a loaded register sits behind a per-thread branch, so the
// compiler's waits for outstanding memory operations stay a tile or more
// behind the loads.  (Measured on the triangle r16: 22.8 us per generation
// with one tile ahead and unaligned loads, 20.4 like this.)
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

// A block's CB bytes are read through one load of a window of ND dwords
// that holds them, from the 4- or 8-byte boundary at or below its first byte:
// unaligned loads cost the vector memory unit about three times as much as
// aligned ones.  A window that would run past the end of the readable bytes
// (in the state's or arena's last tile only) ends there instead.
// sh = offset of the block's first byte in the window.
template <int ND>
struct Window {
    uint32_t d[ND];
    uint32_t sh;
};
// The block's bytes from byte 0 (dword i = bytes 4i..4i+3, NOUT dwords
// used).  STAGES: how many dword moves (by 1, 2, 4) sh may need: 0 when
// sh < 4, 1 when sh < 8, 3 for any sh (a window ended at `lim`).
template <int NSRC, int ND, int NOUT, int STAGES>
__device__ __forceinline__ RawBlock<NSRC> align_window(const Window<ND> &w) {
    RawBlock<NSRC> r;
    const uint32_t h = w.sh >> 2;
    // dwords h.. of the window, moved down by one, two and four dwords as
    // the bits of h say (two-way selects: an indexed pick would go through
    // scratch memory)
    uint32_t x[ND + 1];
#pragma unroll
    for (int i = 0; i < ND; ++i) x[i] = w.d[i];
    x[ND] = 0;
#pragma unroll
    for (int b = 0; b < STAGES; ++b) {
        const int m = 1 << b;
        if (m >= ND) break;
        const bool on = (h >> b) & 1;
#pragma unroll
        for (int i = 0; i <= ND; ++i) x[i] = on ? (i + m <= ND ? x[i + m] : 0u) : x[i];
    }
#pragma unroll
    for (int i = 0; i < NSRC; ++i) r.d[i] = i < NOUT ? alignbyte(x[i + 1], x[i], w.sh) : 0u;  // (uses sh & 3)
    return r;
}
// Whether any thread of the wavefront holds a window with sh >= limit.
template <int ND>
__device__ __forceinline__ bool any_wide(const Window<ND> &w, uint32_t limit) {
    return __builtin_amdgcn_ballot_w64(w.sh >= limit) != 0;
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

// Raw buffer stores into a tile's output: the resource's base is the tile's
// first byte (uniform), its range the whole 32-bit offset space (untyped
// 32-bit data format, as gfx9 buffer resources need for untyped stores).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(uint8_t *base) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, -1, 0x00020000);
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// Stores the CB compact bytes of w at byte offset off of the resource (any
// alignment), as store_cells does.
template <int CBC>
__device__ __forceinline__ void store_cells_buf(const uint32_t (&w)[4], uint32_t CB_, __amdgpu_buffer_rsrc_t r,
                                                uint32_t off) {
    const uint32_t CB = CBC ? uint32_t(CBC) : CB_;
    const u32x2 w01 = {w[0], w[1]}, w23 = {w[2], w[3]};
    if (CB == 16) {
        __builtin_amdgcn_raw_buffer_store_b64(w01, r, off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(w23, r, off + 8, 0, 0);
    } else if (CB > 8) {
        __builtin_amdgcn_raw_buffer_store_b64(w01, r, off, 0, 0);
        uint32_t rem = CB - 8, x = w[2], o = off + 8;
        if (rem >= 4) {
            __builtin_amdgcn_raw_buffer_store_b32(x, r, o, 0, 0);
            o += 4;
            rem -= 4;
            x = w[3];
        }
        if (rem >= 2) {
            __builtin_amdgcn_raw_buffer_store_b16(uint16_t(x), r, o, 0, 0);
            o += 2;
            rem -= 2;
            x >>= 16;
        }
        if (rem) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(x), r, o, 0, 0);
    } else if (CB == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(w01, r, off, 0, 0);
    } else if (CB > 4) {
        __builtin_amdgcn_raw_buffer_store_b32(w[0], r, off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(alignbyte(w[1], w[0], CB - 4), r, off + (CB - 4), 0, 0);
    } else if (CB == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(w[0], r, off, 0, 0);
    } else if (CB >= 2) {
        __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[0]), r, off, 0, 0);
        if (CB == 3) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[0] >> 8), r, off + 1, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b8(uint8_t(w[0]), r, off, 0, 0);
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
    // The window per block (ND dwords from a kAlign-byte boundary), the
    // dwords of block bytes used, and whether a window ended at the readable
    // end can leave the block kAlign or more bytes in.  Blocks of 4, 8 or 16
    // cells start aligned to their size (tiles hold a multiple of CB cells,
    // states start 16-aligned): their window is the block itself.  Blocks of
    // at most 13 cells whose count is known read the dwords from the 4-byte
    // boundary at or below them, so that v_alignbyte alone moves them into
    // place.  Others read 16 or 24 bytes from the 8-byte boundary.
    constexpr bool kAW = CBC == 4 || CBC == 8 || CBC == 16;
    constexpr bool kA4 = !kAW && CBC && CBC <= 13;
    constexpr int ND = kAW ? CBC / 4 : (kA4 ? (CBC + 6) / 4 : ((NSRC == 2 || (CBC && CBC <= 9)) ? 4 : 6));
    constexpr int NOUT = CBC ? (CBC + 3) / 4 : NSRC;
    constexpr uint32_t kAlign = kA4 ? 4 : 8;
    constexpr uint32_t WB = 4 * ND;  // window bytes
    constexpr bool kWide = !kAW && !(CBC && WB - CBC < kAlign);
    // neighbour entries of four tiles in a ring (written by wavefront 0)
    __shared__ uint32_t nbr[4][kLanes];
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    // The halo items and the neighbour entries go to wavefronts that rotate
    // with the work-group, so that no SIMD carries that work for every
    // work-group on the CU.
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid) >> 6, rot = blockIdx.x & 3;
    const bool went = wave == ((rot + 2) & 3);  // the neighbour entries
    const uint32_t hslot = (((wave + 4 - rot) & 3) << 6) | lane;  // this thread's halo position
    const uint32_t K = E.K, CB = E.CB;
    const XcdRange R64 = xcd_range(blockIdx.x, gridDim.x, E.ntiles);
    // tile numbers fit 32 bits (E.ntiles does)
    const uint32_t first = uint32_t(R64.first), end = uint32_t(R64.end), step = uint32_t(R64.step);
    if (first >= end) return;
    // The work-group's tiles are first + i step.  Loads run up to four
    // tiles ahead; past the last tile they read the last tile again (cached).
    // 32-bit arithmetic throughout (a tile holds at least 32 cells, so tile
    // numbers stay below 2^31 and first + (i + 4) step does not wrap); 64-bit
    // compares would need vector registers.
    const uint32_t last = first + (end - 1 - first) / step * step;
    auto clamp = [&](uint32_t i) -> uint32_t {  // the work-group's i-th tile
        return min(first + i * step, last);
    };
    auto entry = [&](uint32_t t, uint32_t l) -> uint32_t {
        return (!BATCH || l < 8) ? E.nbr[uint64_t(t) * 8 + l] : rec[uint64_t(t) * 2 + (l - 8)];
    };

    constexpr uint32_t SR = edge_rec_stride(BPT, HPT);
    for (uint32_t o = tid * 16; o < 16 * SR; o += 256 * 16)
        *reinterpret_cast<uint4 *>(lds_e + o) = make_uint4(0, 0, 0, 0);
    const RuleTables RT = rule_tables(rule);
    // This thread's blocks (the same in every tile).  A thread beyond the
    // tile's blocks takes block number modulo their count again and writes
    // and stores the same values as that block's own thread, so that no load,
    // store or use of a loaded register sits behind a per-thread branch and
    // the compiler's waits for outstanding memory operations count exactly.
    // For j >= 1 a wavefront none of whose threads has a j-th block of its
    // own skips that block altogether (a uniform branch).
    EdgeNbrs nb[BPT];
    uint32_t own[BPT], boff[BPT];
    bool bwave[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        bwave[j] = j == 0 || (wave << 6) + 256 * j < E.nblk;
        const uint32_t bi = (tid + 256 * j) % E.nblk;
        const uint4 w = *reinterpret_cast<const uint4 *>(E.blk + 4 * bi);
        nb[j] = EdgeNbrs{(w.x & 0xFFFFu) * 4, (w.x >> 16) * 4, (w.y & 0xFFFFu) * 4, (w.y >> 16) * 4,
                         (w.z & 0xFFFFu) * 4, (w.z >> 16) * 4, (w.w & 0xFFFFu) * 4, (w.w >> 16) * 4};
        own[j] = bi * 4;
        boff[j] = bi * CB;
    }
    // Halo items: item h is the thread with halo position h % 256, j = h /
    // 256; only wavefronts that hold an item load and write them (a uniform
    // branch).  A thread without an item loads its own block's window and
    // writes to a record nobody reads (past the record of zeros).
    uint32_t hdir[HPT], hoff[HPT], hrec[HPT];
    bool hwave[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const uint32_t h = hslot + 256 * j;
        const bool ok = h < E.nhalo;
        const uint32_t w0 = ok ? E.halo[2 * h] : 0u, w1 = ok ? E.halo[2 * h + 1] : 0u;
        hdir[j] = ok ? (w0 >> 29) : 8u;  // 8: no item
        hoff[j] = (w0 & 0x1FFFFFFFu) * CB;
        hrec[j] = (ok ? (w1 & 0xFFFFu) : E.nblk + h + 1) * 4;
        hwave[j] = (hslot & ~63u) + 256 * j < E.nhalo;
    }

    // The loads of a tile, issued two tiles ahead of its rule.
    struct Pending {
        Window<ND> raw[BPT], hraw[HPT];
        bool hok[HPT];
        bool tail;  // the tile's own windows may end at the readable end
        const uint8_t *src;  // the state the tile belongs to
        uint8_t *dst;
        uint32_t local, lim;  // local tile number, readable bytes from src
    };
    // one window (32-bit offset from the state, any block of it): from the
    // 8-byte boundary at or below the block, or ending at the readable end
    auto window = [&](const uint8_t *src, uint32_t off, uint32_t lim, bool may_end) -> Window<ND> {
        Window<ND> w;
        if (kAW) {
            w.sh = 0;
            constexpr int kB = kAW ? CBC : 4;  // (the branch is not taken otherwise)
            __builtin_memcpy(w.d, __builtin_assume_aligned(src + off, kB), kB);
            return w;
        }
        // (states and arenas start 16-aligned, so the offset alone gives the
        // alignment)
        const uint32_t sh = off & (kAlign - 1);
        uint32_t s = off - sh;
        if (may_end) s = s > lim - WB ? lim - WB : s;
        w.sh = off - s;
        __builtin_memcpy(w.d, src + s, WB);
        return w;
    };
    auto prefetch = [&](Pending &P, uint32_t t, const uint32_t *e) {
        uint64_t base = 0;
        if (BATCH) {
            base = uint64_t(__builtin_amdgcn_readfirstlane(e[8])) << 4;
            P.local = __builtin_amdgcn_readfirstlane(e[9]) & 0x7FFFFFFFu;
        } else {
            P.local = t;
        }
        P.src = in + base;
        P.dst = out + base;
        const uint64_t room = E.limit - base;  // bytes readable from src
        P.lim = room > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(room);
        const uint32_t toff = P.local * K;
        const bool tail = toff + K > P.lim - WB;  // uniform
        P.tail = tail;
#pragma unroll
        for (int j = 0; j < BPT; ++j)  // (a uniform branch: both sides issue the same loads)
            if (bwave[j]) P.raw[j] = tail ? window(P.src, toff + boff[j], P.lim, true)
                                          : window(P.src, toff + boff[j], P.lim, false);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hwave[j]) {
                const uint32_t nt = e[hdir[j] & 7];
                P.hok[j] = hdir[j] < 8 && nt != kOutside;
                P.hraw[j] = window(P.src, P.hok[j] ? nt * K + hoff[j] : toff + boff[0], P.lim, true);
            }
        }
    };
    auto aligned = [&](const Window<ND> &w, bool may_be_wide) -> RawBlock<NSRC> {
        if (kAW) {
            RawBlock<NSRC> r;
#pragma unroll
            for (int i = 0; i < NSRC; ++i) r.d[i] = i < ND ? w.d[i < ND ? i : 0] : 0u;
            return r;
        }
        if (kWide && may_be_wide && any_wide<ND>(w, kAlign)) return align_window<NSRC, ND, NOUT, 3>(w);
        return align_window<NSRC, ND, NOUT, kA4 ? 0 : 1>(w);
    };
    const EdgeRecs<SR> grid{lds_e};
    // step 1 of a tile: the records of its blocks (kept as rows) and halo blocks
    uint32_t rows[BPT][BS];
    auto records = [&](Pending &P) {
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            if (!bwave[j]) continue;
            unpack_rows<BS, NSRC, SEL>(E, aligned(P.raw[j], P.tail), rows[j]);
            grid.put(own[j], edge_record<BS>(rows[j]));
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hwave[j]) {
                uint32_t hr[BS];
                unpack_rows<BS, NSRC, SEL>(E, aligned(P.hraw[j], true), hr);
                grid.put(hrec[j], edge_record<BS>(hr));
                // an item whose neighbour tile does not exist is a block of zeros
                if (!P.hok[j]) grid.put(hrec[j], make_uint4(0, 0, 0, 0));
            }
        }
    };

    // Start: the entries of the first four tiles (the fourth's stay in a
    // register until the first tile is done), the loads of the first two
    // tiles, the first tile's records.
    Pending P0, P1;
    uint32_t c0 = 0, c1 = 0;
    const uint32_t lslot = lane < kLanes ? lane : 0u;
    if (went) {
        const uint32_t e0 = entry(clamp(0), lslot), e1 = entry(clamp(1), lslot), e2 = entry(clamp(2), lslot);
        c1 = entry(clamp(3), lslot);
        if (lane < kLanes) {
            nbr[0][lane] = e0;
            nbr[1][lane] = e1;
            nbr[2][lane] = e2;
        }
    }
    __syncthreads();
    prefetch(P0, first, nbr[0]);
    prefetch(P1, clamp(1), nbr[1]);
    records(P0);

    // Tile number i: its records are written (visible after the first
    // barrier), P holds the loads of the next tile and Q's registers
    // (consumed) take those of the tile after it; cl receives the entries of
    // the tile four ahead, cw holds those of the tile three ahead.
    uint32_t i = 0;
    auto body = [&](Pending &Q, Pending &P, uint32_t &cl, const uint32_t &cw) -> bool {
        // the tile's output as a buffer resource (its base uniform), so that each
        // store takes the block's 32-bit offset as it is
        const __amdgpu_buffer_rsrc_t gout = out_rsrc(Q.dst + uint64_t(Q.local * K));
        __syncthreads();
        if (went) cl = entry(clamp(i + 4), lslot);
        prefetch(Q, clamp(i + 2), nbr[(i + 2) & 3]);
        // step 2: the rule per block, next states straight to global memory
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            if (!bwave[j]) continue;
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
            store_cells_buf<CBC>(w, CB, gout, boff[j]);
        }
        // the records are read until here; the next tile's come after
        __syncthreads();
        if (went && lane < kLanes) nbr[(i + 3) & 3][lane] = cw;
        ++i;
        if (first + i * step >= end) return false;
        records(P);
        return true;
    };
    for (;;) {
        if (!body(P0, P1, c0, c1)) break;
        if (!body(P1, P0, c1, c0)) break;
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
// against 26.3 in the general form (before loads ran two tiles ahead).  Any
// other plan takes the general form.
struct EdgeSpec {
    uint32_t BS, nsrc, CB, sel;
};
constexpr EdgeSpec kSpecTriangle{4, 4, 9, 0x6387u};
// The same for the other fractals of the batched and served workloads at
// block level 1: the carpet F^{8,3}, the H F^{7,3} and the chandelier-like
// F^{4,3} (whose third block row holds no cell; chandelier r13 at level 5:
// 36.2 -> 31.2 us per generation, H r10 forced into this form 176 -> 172).
constexpr EdgeSpec kSpecCarpet{3, 2, 8, 0x2307u};
constexpr EdgeSpec kSpecH{3, 2, 7, 0x3307u};
constexpr EdgeSpec kSpecChandelier{3, 2, 4, 0x0103u};
// Blocks of 4, 8 or 16 cells (the chandelier-like F^{4,3} and the carpet
// F^{8,3} at block level 1, the full square at level 2): every block starts
// aligned to its size, one aligned load and store each (any selector mask).
constexpr EdgeSpec kSpecFour{3, 2, 4, kAllSel};
constexpr EdgeSpec kSpecEight{3, 2, 8, kAllSel};
constexpr EdgeSpec kSpecSixteen{4, 4, 16, kAllSel};

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
    NBB_EDGES_SPEC(kSpecCarpet);
    NBB_EDGES_SPEC(kSpecH);
    NBB_EDGES_SPEC(kSpecChandelier);
#undef NBB_EDGES_SPEC
#define NBB_EDGES_ALIGNED(P)                                                                                     \
    if (BS == P.BS && nsrc == P.nsrc && E.CB == P.CB)                                                           \
    return launch_edges_s<P.BS, P.nsrc, BATCH, EDGE, RULE, P.CB, kAllSel>(E, in, out, rule, rec, cu_count, caps, st)
    NBB_EDGES_ALIGNED(kSpecFour);
    NBB_EDGES_ALIGNED(kSpecEight);
    NBB_EDGES_ALIGNED(kSpecSixteen);
#undef NBB_EDGES_ALIGNED
    if (BS == 3 && nsrc == 2)
        return launch_edges_s<3, 2, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    if (BS == 3 && nsrc == 4)
        return launch_edges_s<3, 4, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    if (BS == 4 && nsrc == 4)
        return launch_edges_s<4, 4, BATCH, EDGE, RULE>(E, in, out, rule, rec, cu_count, caps, st);
    return hipErrorInvalidValue;
}

}  // namespace nbb
