// Device helpers shared by the kernels of kernels.hip and tiled.hpp: integer
// division by invariants, byte funnel shifts, the XCD-aware tile ranges, the
// tiled step's prefetch, rule evaluation per block and block stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.hpp"

namespace nbb {


static constexpr uint32_t kOutside = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t udiv(const UDiv &u, uint32_t a) {
    uint32_t t = __umulhi(a, u.m);
    return (t + ((a - t) >> u.s1)) >> u.s2;
}

__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

// Bit j of the 4-bit nibble -> byte j (value 0 or 1) of a dword.
__device__ __forceinline__ uint32_t nibble_to_bytes(uint32_t nib) {
    return __umul24(nib, 0x00204081u) & 0x01010101u;
}

// Work-group -> work-item mapping that keeps a contiguous range of items on
// each XCD.  Work-groups are dispatched round-robin over the 8 XCDs
// (blockIdx % 8), so group x of every 8 gets the x-th slice of the items and
// walks it in order; neighbouring items then share that XCD's L2.
struct XcdRange {
    uint64_t first, end, step;
};
// With `sub` workers per work-group (worker w of group wg), the XCD's slice
// is shared by all workers of its work-groups.
__device__ __forceinline__ XcdRange xcd_range(uint32_t wg, uint32_t G, uint64_t T, uint32_t w = 0,
                                              uint32_t sub = 1) {
    XcdRange r;
    if (G >= 8) {
        uint32_t x = wg & 7, slot = (wg >> 3) * sub + w;
        uint32_t cnt = (G - x + 7) >> 3;
        uint64_t before = uint64_t(x) * (G >> 3) + min(x, G & 7);
        uint64_t start = T * before / G;
        r.end = T * (before + cnt) / G;
        r.first = start + slot;
        r.step = uint64_t(cnt) * sub;
    } else {
        r.first = uint64_t(wg) * sub + w;
        r.end = T;
        r.step = uint64_t(G) * sub;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Compact step, tiled: the kernel and its helpers (the kernel's comment
// describes the scheme).
// ---------------------------------------------------------------------------
// Registers holding the next tile's input while the current one computes.
template <int CPT, int HPT>
struct TilePrefetch {
    uint4 v[CPT];      // 16 compact bytes per chunk
    uint4 e[CPT][2];   // their 16 LDS-box offsets (u16)
    uint32_t halo[HPT];
};

// Loads tile t (local index within the state array `in` of cells `cells`)
// and its halo.  `tail`: the tile holds the last cell of an array whose
// length is not a multiple of 16, so its last chunk may not be read whole.
// The scatter offsets depend only on the tile's phase (t K mod 16), and a
// worker's tiles usually share it (consecutive tiles of a worker are a
// multiple of 16 tiles apart), so with KEEP they are reloaded only when the
// phase differs from `pf_ph`, the phase of the offsets held in pf.e.  (Over
// the tiles of a batch, measured slower: the batched step reloads always.)
template <int TEAM, int CPT, int HPT, bool KEEP>
__device__ __forceinline__ void tile_prefetch(const TileParams &T, const uint8_t *__restrict__ in,
                                              uint32_t t, bool tail, uint32_t cells, const uint32_t *nb,
                                              const uint32_t *hsrc, TilePrefetch<CPT, HPT> &pf, uint32_t &pf_ph) {
    const uint32_t tid = threadIdx.x % TEAM;
    const uint32_t B = t * T.K;
    const uint32_t ph = B & 15;
    const uint32_t nchunks = (ph + T.K + 15) >> 4;
    const uint8_t *gin = in + (B & ~15u);  // uniform; chunk c at gin + 16 c
    const uint16_t *lut = T.lut0p + ph * T.lut0_stride;
    const bool reload = !KEEP || ph != pf_ph;  // uniform
    pf_ph = ph;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const uint32_t c = tid + TEAM * j;
        if (c < nchunks) {
            if (!tail || c + 1 < nchunks) {
                pf.v[j] = *reinterpret_cast<const uint4 *>(gin + 16 * c);
            } else {
                uint32_t v[4] = {0, 0, 0, 0};
                const uint32_t nb_ = cells & 15;
                for (uint32_t b = 0; b < nb_; ++b) v[b >> 2] |= uint32_t(gin[16 * c + b]) << (8 * (b & 3));
                pf.v[j] = make_uint4(v[0], v[1], v[2], v[3]);
            }
            if (reload) {
                pf.e[j][0] = *reinterpret_cast<const uint4 *>(lut + 16 * c);
                pf.e[j][1] = *reinterpret_cast<const uint4 *>(lut + 16 * c + 8);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const uint32_t src = hsrc[j];  // kOutside: this thread has no j-th halo cell
        const uint32_t nt = src != kOutside ? nb[src >> 29] : kOutside;
        pf.halo[j] = nt != kOutside ? in[nt * T.K + (src & 0x1FFFFFFFu)] : 0u;
    }
}

// The B3/S23 rule word.
constexpr uint32_t kRuleB3S23 = (1u << 3) | ((1u << 2 | 1u << 3) << 16);

// The rule as two byte tables for v_perm: byte c of born (c = 0..7) is the
// birth bit for c live neighbours, byte c of surv the survival bit; counts
// 0-3 sit in the low dword, 4-7 in the high one.  A count of 8 selects a sign
// byte of the table (0, as every table byte is 0 or 1), so the tables serve
// exactly the rules without birth or survival at 8 (`perm`).
struct RuleTables {
    uint32_t born_lo, born_hi, surv_lo, surv_hi;
    bool perm;
};
__device__ __forceinline__ RuleTables rule_tables(uint32_t rule) {
    RuleTables t{0, 0, 0, 0, (rule & ((1u << 8) | (1u << 24))) == 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        t.born_lo |= ((rule >> c) & 1u) << (8 * c);
        t.born_hi |= ((rule >> (c + 4)) & 1u) << (8 * c);
        t.surv_lo |= ((rule >> (c + 16)) & 1u) << (8 * c);
        t.surv_hi |= ((rule >> (c + 20)) & 1u) << (8 * c);
    }
    return t;
}

// Next states of one block (a BS x BS square whose CB fractal cells are
// consecutive in compact order), one byte per position: row r of the block
// in next[r], byte c = column c (bytes past BS and rows past BS are
// unspecified or 0).  The window is BS+2 rows of the LDS box starting one row
// up and one column left of the block, read as two dwords per row; byte c of
// H is the 3-sum of window columns c..c+2, so H[r] + H[r+1] + H[r+2] - self
// is the live-neighbour count of every position of block row r at once.
//   RULE 0, B3/S23: born with 3, survives with 2 or 3, i.e. alive next iff
//   (neighbours | self) == 3, one v_perm for four positions (selector 3 picks
//   the table's 1, every other value 0..9 a zero byte);
//   RULE 1, rules without birth or survival at 8: two v_perm look up the
//   birth and the survival byte of four positions at once and self picks
//   between them;
//   RULE 2, any rule: each byte indexes the rule word (neighbours + 16 * self).
// ROWS < BS: only the block's first ROWS rows hold fractal cells (e.g. the
// chandelier's 3x3 blocks, whose third row is empty), so only ROWS + 2 window
// rows are read and ROWS rows evaluated.
template <int BS, int RULE, bool EDGE, int ROWS = BS>
__device__ __forceinline__ void block_rows(const uint32_t *box32, uint32_t W4, uint32_t base, uint32_t rule,
                                           const RuleTables &RT, uint32_t (&next)[4]) {
    const uint32_t a0 = base >> 2, sh = base & 3;
    uint32_t lo[BS + 2], hi[BS + 2], C[BS + 2], H[BS + 2];
#pragma unroll
    for (int rr = 0; rr < ROWS + 2; ++rr) {
        const uint32_t d0 = box32[a0 + rr * W4], d1 = box32[a0 + rr * W4 + 1];
        if (BS == 4) {            // corner column is 4-aligned
            lo[rr] = d0;
            hi[rr] = d1;
        } else {
            lo[rr] = alignbyte(d1, d0, sh);   // window columns 0..3
            hi[rr] = d1 >> (8 * sh);          // window columns 4..
        }
        if (BS == 2) {
            C[rr] = lo[rr] >> 8;
            H[rr] = lo[rr] + C[rr] + (lo[rr] >> 16);
        } else {
            C[rr] = alignbyte(hi[rr], lo[rr], 1);
            H[rr] = lo[rr] + C[rr] + alignbyte(hi[rr], lo[rr], 2);
        }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        if (rr >= ROWS) {  // rows past ROWS hold no fractal cell
            next[rr] = 0;
            continue;
        }
        const uint32_t self = C[rr + 1];
        // live neighbours per byte: the 3x3 sum minus self, or the cells
        // above and below plus the left and right ones
        uint32_t n;
        if (EDGE)
            n = C[rr] + C[rr + 2] + lo[rr + 1] +
                (BS == 2 ? lo[rr + 1] >> 16 : alignbyte(hi[rr + 1], lo[rr + 1], 2));
        else
            n = H[rr] + H[rr + 1] + H[rr + 2] - self;
        if (RULE == 0) {
            next[rr] = __builtin_amdgcn_perm(0u, 0x01000000u, n | self);
        } else if (RULE == 1) {
            const uint32_t born = __builtin_amdgcn_perm(RT.born_hi, RT.born_lo, n);
            const uint32_t surv = __builtin_amdgcn_perm(RT.surv_hi, RT.surv_lo, n);
            const uint32_t smask = __builtin_amdgcn_perm(0u, 0x0000FF00u, self);  // 0xFF where alive
            next[rr] = (born & ~smask) | (surv & smask);
        } else {
            // v_bfe takes its offset from the low 5 bits of the operand, and
            // byte c of I (<= 24) is exactly those bits of I >> 8c
            const uint32_t I = n + (self << 4);
            uint32_t v = __builtin_amdgcn_ubfe(rule, I, 1);
#pragma unroll
            for (int cc = 1; cc < BS; ++cc) v |= __builtin_amdgcn_ubfe(rule, I >> (8 * cc), 1) << (8 * cc);
            next[rr] = v;
        }
    }
}

__device__ __forceinline__ void store_u8(uint8_t *p, uint32_t v) { *p = uint8_t(v); }
__device__ __forceinline__ void store_u16(uint8_t *p, uint32_t v) {
    const uint16_t h = uint16_t(v);
    __builtin_memcpy(p, &h, 2);
}
__device__ __forceinline__ void store_u32(uint8_t *p, uint32_t v) { __builtin_memcpy(p, &v, 4); }
__device__ __forceinline__ void store_u64(uint8_t *p, uint32_t v0, uint32_t v1) {
    const uint64_t v = uint64_t(v1) << 32 | v0;
    __builtin_memcpy(p, &v, 8);
}

// Gathers the block's member bytes into compact order with v_perm and stores
// its CB next states at p (any alignment: gfx950 global stores need none).
// Blocks of 5 to 7 cells are written as two overlapping 4-byte stores of the
// same lane (the overlap gets the same bytes twice; blocks of different
// lanes never overlap).  CB is uniform, so the choice below is scalar
// branches only.
template <int BS>
__device__ __forceinline__ void block_store(const TileParams &T, const uint32_t (&next)[4], uint8_t *p) {
    uint32_t w[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        w[d] = __builtin_amdgcn_perm(next[1], next[0], T.pack01[d]);
        if (BS >= 3) w[d] |= __builtin_amdgcn_perm(next[3], next[2], T.pack23[d]);
    }
    const uint32_t CB = T.CB;  // 1..16 bytes
    if (CB == 16) {
        store_u64(p, w[0], w[1]);
        store_u64(p + 8, w[2], w[3]);
    } else if (CB > 8) {
        // (an overlapping second 8-byte store measured slower than the
        // pieces for the 9-cell blocks of the triangle)
        store_u64(p, w[0], w[1]);
        uint32_t r = CB - 8, x = w[2];  // 1..7
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

}  // namespace nbb
