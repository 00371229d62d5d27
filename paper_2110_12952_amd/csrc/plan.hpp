// Host-side description of an NBB fractal and every table the kernels use.
// Pure C++ (no HIP calls): the C-ABI layer uploads these tables.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "params.hpp"

namespace nbb {

UDiv make_udiv(uint32_t d);
uint32_t udiv_apply(const UDiv &u, uint32_t a);  // host check of the same formula

struct Fractal {
    uint32_t k = 0, s = 0, r = 0;
    uint64_t n = 0, cells = 0;
    int32_t ox[kMaxK] = {}, oy[kMaxK] = {};
    uint8_t hl[256];  // a + s*b -> replica id or 0xFF
};

// Checks the arguments of nbb_create; returns 0 (ok), 1 (invalid) or 2 (range)
// and fills *msg on failure.
int validate_fractal(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r, Fractal *f,
                     std::string *msg);

// lambda and nu at `levels` levels (levels <= r), plain digit loops.
void lambda_levels(const Fractal &f, uint32_t levels, uint64_t i, int64_t *x, int64_t *y);
int64_t nu_levels(const Fractal &f, uint32_t levels, int64_t x, int64_t y);  // -1 outside

struct MapTables {
    uint32_t jl = 0, jl_top = 0, nchunks_l = 0, jn = 0, jn_top = 0, nchunks_n = 0;
    std::vector<uint32_t> lam;  // low table then top table
    uint32_t lam_top_off = 0;
    std::vector<uint16_t> nu;   // low table then top table
    uint32_t nu_top_off = 0;
};
void build_map_tables(const Fractal &f, MapTables *t);

struct TilePlan {
    bool ok = false;
    uint32_t team = 256;  // threads per tile: 256 (work-group) or 64 (wavefront)
    uint32_t m = 0, S = 0, K = 0, W = 0, q = 0, BS = 0, CB = 0, nblk = 0;
    uint32_t rows = 0;  // box rows read by the rule (<= S + 2)
    uint32_t brows = 0;  // rows of a block that hold cells (the first brows rows)
    uint32_t box_bytes = 0, lds_total = 0;
    uint32_t rm = 0, Sc = 0, lut0_stride = 0, dummy = 0;
    uint8_t bid[16];
    uint32_t pack01[4] = {}, pack23[4] = {};  // see TileParams
    uint64_t ntiles = 0;
    std::vector<uint16_t> lut0;   // phase 0, K entries
    std::vector<uint16_t> lut0p;  // 16 phase copies
    std::vector<uint16_t> lut1;
    std::vector<uint32_t> halo_src, halo_dst;
    std::vector<uint32_t> nbr;    // 8 per tile: nu_{r-m} of the neighbouring coarse coordinates
    // Blocked layout (each tile stored as its S x S square): position y*S + x
    // of local cell j, and per row y and 4-column group c a dword with byte b
    // = 1 where (4c + b, y) is a fractal cell (S rows of ceil(S/4) dwords).
    std::vector<uint32_t> blk_pos, blk_mask;
};
// True if the tiled step supports this fractal (2 <= s <= 4, r >= 1).
bool tiled_supported(const Fractal &f);
// Largest usable tile level, then reduced while fewer than `min_tiles` tiles.
uint32_t auto_tile_level(const Fractal &f);
// Builds the plan at tile level m (1 <= m <= r) for teams of `team` threads
// per tile (256 or 64); false if it does not fit.
bool build_tile_plan(const Fractal &f, uint32_t m, TilePlan *p, std::string *msg, uint32_t team = 256);

// The edge-record form of the tiled step (EdgeParams) at tile level m: each
// block's eight neighbouring records, halo items and v_perm selectors.  Uses
// the neighbour table of the tile plan at the same level.
struct EdgePlan {
    bool ok = false;
    uint32_t m = 0, q = 0, S = 0, K = 0, BS = 0, CB = 0, G = 0, nblk = 0, nhalo = 0;
    uint32_t nsrc = 0;      // dwords per block load: 2 (3 x 3 blocks of at most 8 cells) or 4
    uint32_t nrec = 0;      // records: the blocks, the halo items and one of zeros
    uint32_t rec_bytes = 0; // 16 bytes per record, rounded up to 4 records
    uint32_t unpack01[4] = {}, unpack23[4] = {}, pack01[4] = {}, pack23[4] = {};
    std::vector<uint32_t> blk;   // 4 per block, see EdgeParams
    std::vector<uint32_t> halo;  // 2 per halo item, see EdgeParams
    std::vector<int32_t> blk_xy; // 2 per block: its grid coordinates (X, Y) in [0, G)
    std::vector<int32_t> halo_xy; // 2 per halo item: ring coordinates in [-1, G]
};
// false (with *msg) if the form does not apply at this level: tiles below
// 2 loads' width, more than 1024 blocks or more than 512 halo items.
bool build_edge_plan(const Fractal &f, uint32_t m, EdgePlan *p, std::string *msg);

// Several generations per launch (temporal blocking) for small instances: a
// work-group holds tile t's S x S square and a ring of depth h around it (the
// cells of the eight neighbour tiles within h of the square) as a box of side
// B = S + 2h in LDS, steps the box `gens` <= h times there, and writes back
// the tile's own cells, which stay exact because a generation corrupts at
// most one more ring of the box's border.  Box row y, column x (pitch P bytes,
// a multiple of 4) = embedded (x - h, y - h) relative to the tile's corner.
struct TemporalPlan {
    bool ok = false;
    uint32_t m = 0, S = 0, K = 0, h = 0, B = 0, P = 0;
    uint32_t box_bytes = 0;  // B * P, a multiple of 16
    uint32_t lds = 0;        // three boxes: two state copies and the member mask
    uint64_t ntiles = 0;
    std::vector<uint32_t> self;  // K entries: box offset of local cell j
    std::vector<uint32_t> halo;  // 2 per item: direction << 29 | local index, box offset
    std::vector<uint32_t> nbr;   // 8 per tile, as the tile plan's
};
// false (with *msg) unless 2 <= s <= 4, 1 <= m <= r, 1 <= h <= S and the three
// boxes fit `lds_limit` bytes.
bool build_temporal_plan(const Fractal &f, uint32_t m, uint32_t h, uint32_t lds_limit, TemporalPlan *p,
                         std::string *msg);

// Matrix-core maps: A for lambda and Anu for nu (16 x 32*ktiles int8 each),
// see MfmaLambda in params.hpp.  ktiles == 0 when unsupported (r*k > 192 or
// n > 2^28).
struct MfmaTables {
    uint32_t ktiles = 0;
    std::vector<int8_t> A, Anu;
};
void build_mfma_tables(const Fractal &f, MfmaTables *t);

struct BoxTables {
    uint32_t L = 0, SL = 0, LW = 0, NH = 0;
    std::vector<uint32_t> low;
    std::vector<uint8_t> high;
};
void build_box_tables(const Fractal &f, BoxTables *b);

uint64_t box_pitch(const Fractal &f);

}  // namespace nbb
