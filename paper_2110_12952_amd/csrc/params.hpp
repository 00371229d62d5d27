// Launch parameter blocks shared by the host plan builder and the HIP kernels.
// Plain structs passed by value as kernel arguments, so every field is uniform
// across a wavefront and lives in scalar registers / the kernel-argument
// segment.
#pragma once
#include <stdint.h>

namespace nbb {

// Division by a run-time invariant d with one multiply-high (Granlund &
// Montgomery, "Division by invariant integers using multiplication",
// PLDI 1994, fig. 4.1): q = (t + ((a - t) >> s1)) >> s2, t = mulhi(a, m).
// Exact for every 32-bit a and 1 <= d < 2^32.
struct UDiv {
    uint32_t m, s1, s2, d;
};

constexpr int kMaxK = 256;  // k <= s^2 <= 256

// Tables and constants for the maps lambda / nu (section 3) and for every
// kernel that evaluates them per element.
struct MapParams {
    uint32_t k, s, r;
    uint32_t n;          // s^r (n + 1 < 2^31)
    uint32_t cells_m1;   // k^r - 1
    UDiv divk, divs;
    // lambda in chunks of jl levels: table of k^jl packed (x | y << 16) for the
    // low chunks, and one of k^jl_top entries for the most significant chunk.
    uint32_t jl, jl_top, nchunks_l;
    uint32_t kl, sl;     // k^jl, s^jl
    UDiv divkl;
    uint32_t lam_top_off;  // offset (entries) of the top table in lam_lut
    // nu in chunks of jn levels: (s^jn)^2 table, entry = local compact index
    // or 0xFFFF, indexed yc * s^jn + xc; the top chunk has its own table.
    uint32_t jn, jn_top, nchunks_n;
    uint32_t sn, kn, sn_top;
    UDiv divsn;
    uint32_t nu_top_off;
    const uint32_t *lam_lut;
    const uint16_t *nu_lut;
    const uint8_t *ox;   // replica offsets (k entries)
    const uint8_t *oy;
    const uint8_t *hl;   // digit pair a + s*b -> replica id, 0xFF if none
};

// lambda as in the paper's per-thread map (section 3.1: one term per level)
// and its matrix-core form: the per-level sum sum_mu o_{d_mu} s^mu as an int8
// contraction D = A B with B[(mu, j)][item] = [d_mu(item) == j] (one-hot
// digits) and A[row][(mu, j)] = 7-bit plane p of o_j.c * s^mu; rows 0-3 hold
// the four x planes, rows 4-7 the four y planes (coordinates < 2^28).
// nu the same way: B[(mu, j)][item] = [H_mu(item) == j] (one-hot replica
// ids of the digit pairs) and Anu[p][(mu, j)] = 7-bit plane p of j k^mu, rows
// 0-4 (indices < 2^32 need five planes).
struct MfmaLambda {
    uint32_t ktiles;        // K = 32 * ktiles >= r * k
    const int8_t *A;        // 16 x (32 * ktiles), row-major
    const int8_t *Anu;      // 16 x (32 * ktiles), row-major
};

// The tiled compact step: a tile is an aligned run of K = k^m compact cells,
// i.e. one level-m copy of the fractal occupying an S x S block (S = s^m) of
// the box.  A work-group stages the tile and the neighbour cells that touch
// it in an LDS box of (S + 2) rows by W bytes, then evaluates the rule per
// level-q block (side BS = s^q, CB = k^q cells, consecutive in compact order).
struct TileParams {
    uint32_t team;        // threads per tile: 256 (work-group) or 64 (wavefront)
    uint32_t m, S, K, W;
    uint32_t q, BS, CB;   // block level, block side s^q, cells per block k^q
    uint32_t nblk;        // k^(m-q) blocks per tile
    uint32_t brows;       // rows of a block that hold cells (its first brows rows)
    uint32_t box_bytes;   // LDS box allocation
    uint32_t lds_total;   // LDS per team
    uint32_t rm;          // coarse levels r - m
    uint32_t ntiles;      // k^(r-m)
    uint32_t Sc;          // s^(r-m)
    uint32_t halo_count;
    uint32_t cells;       // k^r (<= 2^32 - 1)
    uint32_t lut0_stride; // entries per phase copy of lut0
    uint32_t dummy;       // a never-read LDS byte that absorbs writes of cells outside the tile
    const uint16_t *lut0p;   // 16 phase copies: copy p entry j = box offset of local cell j - p
                             // (dummy where j - p is not a cell of the tile)
    const uint16_t *lut1;    // box offset of the window corner of each block
    const uint32_t *halo_src;
    const uint32_t *halo_dst;
    const uint32_t *nbr;     // 8 neighbour tiles per tile (0xFFFFFFFF = none)
    const uint32_t *blk_pos;   // blocked layout: y*S + x of local cell j
    const uint32_t *blk_mask;  // blocked layout: member bytes per row and 4-column group
    UDiv divK, divS;           // division by K and by S
    // v_perm selectors that gather a block's next states, one byte per
    // block position (row r in a dword, byte c = column c), into compact
    // order: output dword d = perm(row1, row0, pack01[d]) | perm(row3, row2,
    // pack23[d]); selector 12 gives a zero byte.
    uint32_t pack01[4], pack23[4];
};

// The edge-record form of the tiled step.  The tile is cut into the same
// level-q blocks (side BS, CB cells, consecutive in compact order) placed on a
// G x G grid (G = S / BS), with a ring of one block around it for the facing
// blocks of the eight neighbour tiles (the halo items).  Each thread loads its
// block's CB bytes into registers, unpacks them into BS row dwords (byte c of
// row r = cell (c, r) of the block, 0 where the block has no cell) and writes
// the block's edges (top row, bottom row, left column, right column; column
// dword: byte r = row r) as its record in four LDS dword arrays, 16 bytes per
// record in all.  Records are numbered in block order (block b is record b,
// halo item h record nblk + h, the last one all zeros), so the lanes of a
// wavefront write consecutive dwords.  A block's 3x3-window ring is then the
// bottom rows of the three records above it, the top rows of the three below
// and the facing columns of its left and right records, found through the
// block's eight neighbour record numbers (the zero record where the grid has
// no block).
//
// A block's bytes (NSRC dwords of them: 2 for 3 x 3 blocks of at most 8
// cells, else 4) are read through one aligned load of a window that holds
// them: the block itself for blocks of 4, 8 or 16 cells, else a few dwords
// from the 4- or 8-byte boundary below the block; a window that would run
// past `limit` ends at it instead.
struct EdgeParams {
    uint32_t K, CB, nblk, nhalo;
    uint32_t ntiles;        // tiles of the launch (batch tiles for a batch)
    uint32_t rec_bytes;     // 16 bytes per record (four dword arrays), rounded up to 4 records
    uint32_t unpack01[4], unpack23[4];  // v_perm selectors: row r = perm(c1, c0, u01[r]) | perm(c3, c2, u23[r])
    uint32_t pack01[4], pack23[4];      // compact dword d = perm(n1, n0, p01[d]) | perm(n3, n2, p23[d])
    const uint32_t *blk;    // 4 per block: the records left | right << 16, above | below << 16,
                            // above-left | above-right << 16, below-left | below-right << 16
    const uint32_t *halo;   // 2 per item: direction << 29 | local block, record
    const uint32_t *nbr;    // 8 neighbour tiles per tile (0xFFFFFFFF = none)
    uint64_t limit;         // bytes of the input that may be read (the state, or the whole arena)
};

// The edge kernel's instantiation for a plan: blocks and halo items per
// thread (BPT in 1, 2, 4; HPT in 1, 2), false if none fits; its record
// arrays hold 256 (BPT + HPT) + 4 records each, a stride known when it is
// compiled, so that the four arrays are reached through instruction offsets.
inline bool edge_case(uint32_t nblk, uint32_t nhalo, uint32_t *bpt, uint32_t *hpt) {
    const uint32_t b = (nblk + 255) / 256, h = (nhalo + 255) / 256;
    if (b > 4 || h > 2) return false;
    *bpt = b <= 1 ? 1 : (b <= 2 ? 2 : 4);
    *hpt = h <= 1 ? 1 : 2;
    return true;
}
// Most resident work-groups per CU of the edge-record step (0: as many as
// fit) for plans of one block per thread and of more.
struct EdgeCaps {
    int one, more;
};
constexpr uint32_t edge_rec_stride(uint32_t bpt, uint32_t hpt) { return 256 * (bpt + hpt) + 4; }
constexpr uint32_t edge_lds_bytes(uint32_t bpt, uint32_t hpt) { return 16 * edge_rec_stride(bpt, hpt); }

// Temporal blocking (several generations per launch): work-group t holds
// tile t's square and a ring of depth h as a B x B box (pitch P bytes) in
// LDS, three times: two state copies and the member mask.
struct TemporalParams {
    uint32_t K, B, P, h;
    uint32_t box_bytes;     // B * P rounded up to 16
    uint32_t nhalo;
    uint32_t ntiles;
    const uint32_t *self;   // K entries: box offset of local cell j
    const uint32_t *halo;   // 2 per item: direction << 29 | local index, box offset
    const uint32_t *nbr;    // 8 per tile (0xFFFFFFFF = none)
};

// One instance of a batch (device table, sorted by tile0): its state starts
// at byte 16 * base16 of the arena; its tiles are batch tiles
// [tile0, tile0 + ntiles); nbr is its own 8-per-tile neighbour table.
struct BatchInstance {
    const uint32_t *nbr;
    uint32_t base16;
    uint32_t tile0;
    uint32_t ntiles;
    uint32_t tail_partial;  // 1 if k^r is not a multiple of 16
};

// One small instance of a batch stepped in LDS: its state at byte
// 16 * base16 of the arenas, `ntiles` tiles of plan `plan` (an index into the
// launch's plan table) taken `teams` at a time, its own neighbour table.
struct ResidentInstance {
    const uint32_t *nbr;
    uint32_t base16;
    uint32_t ntiles;
    uint32_t plan;
    uint32_t teams;
};

// Up to 256 words passed by value to a kernel that stores them.
constexpr uint32_t kWordChunk = 256;
struct WordChunk {
    uint32_t v[kWordChunk];
};

// The bounding-box step.  Membership splits into the low L levels (an
// SL x SL bitmap, SL = s^L, one row of LW words per y) and the high r - L
// levels (an NH x NH byte map, NH = s^(r-L)).
struct BoxParams {
    uint32_t n;
    uint32_t SL, LW, NH;
    UDiv divSL;
    uint32_t rows_per_wg;
    uint64_t pitch;
    const uint32_t *low;
    const uint8_t *high;
};

}  // namespace nbb
