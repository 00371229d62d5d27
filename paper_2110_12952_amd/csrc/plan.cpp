// Host-side tables for the compact-fractal kernels.  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cstring>

namespace nbb {

UDiv make_udiv(uint32_t d) {
    UDiv u{};
    u.d = d;
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;  // l = ceil(log2 d)
    uint64_t two_l = uint64_t(1) << l;
    u.m = uint32_t(((uint64_t(1) << 32) * (two_l - d)) / d + 1);
    u.s1 = l < 1 ? l : 1;
    u.s2 = l > 1 ? l - 1 : 0;
    return u;
}

uint32_t udiv_apply(const UDiv &u, uint32_t a) {
    uint32_t t = uint32_t((uint64_t(a) * u.m) >> 32);
    return (t + ((a - t) >> u.s1)) >> u.s2;
}

static uint64_t upow(uint64_t b, uint32_t e, bool *overflow) {
    uint64_t p = 1;
    for (uint32_t i = 0; i < e; ++i) {
        if (p > (uint64_t(1) << 40) / (b ? b : 1)) *overflow = true;
        p *= b;
        if (p > (uint64_t(1) << 40)) {
            *overflow = true;
            p = uint64_t(1) << 40;
        }
    }
    return p;
}

int validate_fractal(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r, Fractal *f,
                     std::string *msg) {
    if (!offsets) {
        *msg = "offsets is NULL";
        return 1;
    }
    if (k == 0) {
        *msg = "k must be at least 1";
        return 1;
    }
    if (s < 2 || s > 16) {
        *msg = "s must lie in [2, 16]";
        return 1;
    }
    if (k > s * s) {
        *msg = "k may not exceed s*s (replicas cannot overlap)";
        return 1;
    }
    Fractal g;
    std::memset(g.hl, 0xFF, sizeof(g.hl));
    for (uint32_t j = 0; j < k; ++j) {
        int32_t a = offsets[2 * j], b = offsets[2 * j + 1];
        if (a < 0 || b < 0 || a >= int32_t(s) || b >= int32_t(s)) {
            *msg = "replica offset " + std::to_string(j) + " lies outside [0,s)^2";
            return 1;
        }
        if (g.hl[a + s * b] != 0xFF) {
            *msg = "replica offset " + std::to_string(j) + " repeats an earlier one";
            return 1;
        }
        g.hl[a + s * b] = uint8_t(j);
        g.ox[j] = a;
        g.oy[j] = b;
    }
    bool of = false;
    uint64_t n = upow(s, r, &of);
    uint64_t cells = upow(k, r, &of);
    if (of || cells > 0xFFFFFFFFull || n + 1 > 0x7FFFFFFFull) {
        *msg = "level too large: need k^r <= 2^32-1 and s^r + 1 <= 2^31-1";
        return 2;
    }
    g.k = k;
    g.s = s;
    g.r = r;
    g.n = n;
    g.cells = cells;
    *f = g;
    return 0;
}

void lambda_levels(const Fractal &f, uint32_t levels, uint64_t i, int64_t *x, int64_t *y) {
    int64_t px = 0, py = 0, scale = 1;
    for (uint32_t mu = 0; mu < levels; ++mu) {
        uint64_t d = i % f.k;
        i /= f.k;
        px += f.ox[d] * scale;
        py += f.oy[d] * scale;
        scale *= f.s;
    }
    *x = px;
    *y = py;
}

int64_t nu_levels(const Fractal &f, uint32_t levels, int64_t x, int64_t y) {
    int64_t side = 1;
    for (uint32_t mu = 0; mu < levels; ++mu) side *= f.s;
    if (x < 0 || y < 0 || x >= side || y >= side) return -1;
    int64_t idx = 0, w = 1;
    for (uint32_t mu = 0; mu < levels; ++mu) {
        uint32_t h = f.hl[(x % f.s) + f.s * (y % f.s)];
        if (h == 0xFF) return -1;
        idx += int64_t(h) * w;
        w *= f.k;
        x /= f.s;
        y /= f.s;
    }
    return idx;
}

static uint64_t ipow64(uint64_t b, uint32_t e) {
    uint64_t p = 1;
    while (e--) p *= b;
    return p;
}

void build_map_tables(const Fractal &f, MapTables *t) {
    // lambda chunk: k^jl <= 4096 entries (two tables <= 32 KB of LDS), s^jl <= 32768
    // so x, y fit 16 bits.
    uint32_t jl = 1;
    while (ipow64(f.k, jl + 1) <= 4096 && ipow64(f.s, jl + 1) <= 32768 && jl + 1 <= std::max(f.r, 1u))
        ++jl;
    t->jl = jl;
    t->nchunks_l = f.r == 0 ? 0 : (f.r + jl - 1) / jl;
    t->jl_top = f.r == 0 ? 0 : f.r - (t->nchunks_l - 1) * jl;
    uint64_t kl = ipow64(f.k, jl), kt = ipow64(f.k, t->jl_top);
    t->lam.assign(kl + kt, 0);
    for (uint64_t i = 0; i < kl; ++i) {
        int64_t x, y;
        lambda_levels(f, jl, i, &x, &y);
        t->lam[i] = uint32_t(x) | (uint32_t(y) << 16);
    }
    t->lam_top_off = uint32_t(kl);
    for (uint64_t i = 0; i < kt; ++i) {
        int64_t x, y;
        lambda_levels(f, t->jl_top, i, &x, &y);
        t->lam[kl + i] = uint32_t(x) | (uint32_t(y) << 16);
    }
    // nu chunk: (s^jn)^2 <= 8192 entries, k^jn <= 65535 (0xFFFF = outside).
    uint32_t jn = 1;
    while (ipow64(f.s, 2 * (jn + 1)) <= 8192 && ipow64(f.k, jn + 1) <= 65535 && jn + 1 <= std::max(f.r, 1u))
        ++jn;
    t->jn = jn;
    t->nchunks_n = f.r == 0 ? 0 : (f.r + jn - 1) / jn;
    t->jn_top = f.r == 0 ? 0 : f.r - (t->nchunks_n - 1) * jn;
    uint64_t sn = ipow64(f.s, jn), st = ipow64(f.s, t->jn_top);
    t->nu.assign(sn * sn + st * st, 0xFFFF);
    for (uint64_t yc = 0; yc < sn; ++yc)
        for (uint64_t xc = 0; xc < sn; ++xc) {
            int64_t v = nu_levels(f, jn, int64_t(xc), int64_t(yc));
            t->nu[yc * sn + xc] = v < 0 ? 0xFFFF : uint16_t(v);
        }
    t->nu_top_off = uint32_t(sn * sn);
    for (uint64_t yc = 0; yc < st; ++yc)
        for (uint64_t xc = 0; xc < st; ++xc) {
            int64_t v = nu_levels(f, t->jn_top, int64_t(xc), int64_t(yc));
            t->nu[sn * sn + yc * st + xc] = v < 0 ? 0xFFFF : uint16_t(v);
        }
}

bool tiled_supported(const Fractal &f) { return f.s >= 2 && f.s <= 4 && f.r >= 1; }

static uint32_t box_pitch_bytes(uint32_t S) { return (S + 2 + 3) & ~3u; }
static uint32_t box_alloc_bytes(uint32_t S) { return (S + 2) * box_pitch_bytes(S) + 8; }

// LDS budget of the tile box: keeps several work-groups resident per CU.
static const uint32_t kBoxBudget = 32 * 1024;
// LDS per CU on gfx950 and the work-groups of 256 threads one CU holds at
// most (eight waves per SIMD).
static const uint32_t kLdsPerCU = 160 * 1024;
static const uint32_t kMaxGroupsPerCU = 8;

static uint32_t block_level(const Fractal &f, uint32_t m);

// Part of the (S+2)-square box that the rule evaluation reads: rows below
// `rows` and columns below `cols`.  Block b (side BS, level q) reads the BS+2
// rows from Y*BS and two dwords per row from column (X*BS) & ~3, (X, Y) =
// lambda_{m-q}(b).  Fractals whose members never reach the bottom or right
// part of their square (e.g. every y digit in {0, 1}) get a shorter or
// narrower box; halo cells outside it are never read and are not staged.
static void box_extent(const Fractal &f, uint32_t m, uint32_t *rows, uint32_t *cols) {
    const uint32_t q = block_level(f, m), BS = uint32_t(ipow64(f.s, q));
    const uint64_t nb = ipow64(f.k, m - q);
    uint32_t rmax = 0, cmax = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        int64_t X, Y;
        lambda_levels(f, m - q, b, &X, &Y);
        rmax = std::max(rmax, uint32_t(Y * BS + BS + 2));
        cmax = std::max(cmax, uint32_t(((X * BS) & ~int64_t(3)) + 8));
    }
    *rows = rmax;
    *cols = cmax;
}
static uint32_t trimmed_box_bytes(const Fractal &f, uint32_t m) {
    uint32_t rows, cols;
    box_extent(f, m, &rows, &cols);
    return rows * ((cols + 3) & ~3u) + 8;
}
// Below this many tiles a smaller tile level is preferred for parallelism.
static const uint64_t kMinTiles = 512;

// Blocks evaluated per thread: 4x4 squares (two levels) for s = 2 when the
// tile allows, s x s squares (one level) otherwise.
static uint32_t block_level(const Fractal &f, uint32_t m) { return (f.s == 2 && m >= 2) ? 2 : 1; }

static bool fits_group(const Fractal &f, uint32_t m) {
    const uint64_t S = ipow64(f.s, m), K = ipow64(f.k, m);
    return S <= 250 && K + 30 <= 2 * 16 * 256 && ipow64(f.k, m - block_level(f, m)) <= 4 * 256 &&
           trimmed_box_bytes(f, m) <= kBoxBudget;
}

uint32_t auto_tile_level(const Fractal &f) {
    if (!tiled_supported(f)) return 0;
    uint32_t m = 1;
    while (m + 1 <= f.r && fits_group(f, m + 1)) ++m;
    while (m > 1 && ipow64(f.k, f.r - m) < kMinTiles) --m;
    return m;
}

// LDS bank model: 32 banks of 4 bytes, 32 lanes served per cycle; an
// instruction costs, per half-wave, the largest number of distinct dwords that
// fall in one bank.  Used to pick the box pitch for a tile shape: the byte
// scatter of compact cells (lane c writes byte b of 16-byte chunk c) and the
// two-dword window reads of the blocks.
static uint64_t bank_cost(const uint32_t *addr, int lanes) {
    uint64_t cost = 0;
    for (int g = 0; g < lanes; g += 32) {
        uint32_t dw[32];
        int nd = 0;
        for (int l = g; l < lanes && l < g + 32; ++l) {
            uint32_t d = addr[l] >> 2;
            bool seen = false;
            for (int e = 0; e < nd; ++e) seen |= dw[e] == d;
            if (!seen) dw[nd++] = d;
        }
        uint32_t per_bank[32] = {};
        uint32_t worst = 0;
        for (int e = 0; e < nd; ++e) worst = std::max(worst, ++per_bank[dw[e] & 31]);
        cost += worst;
    }
    return cost;
}

static uint64_t box_pitch_cost(const Fractal &f, uint32_t m, uint32_t q, uint32_t W) {
    const uint32_t K = uint32_t(ipow64(f.k, m)), BS = uint32_t(ipow64(f.s, q));
    std::vector<uint32_t> pos(K);
    for (uint32_t i = 0; i < K; ++i) {
        int64_t x, y;
        lambda_levels(f, m, i, &x, &y);
        pos[i] = uint32_t((y + 1) * W + (x + 1));
    }
    uint64_t cost = 0;
    uint32_t addr[64];
    const uint32_t nch = (K + 15) / 16;
    for (uint32_t c0 = 0; c0 < nch; c0 += 64)
        for (uint32_t b = 0; b < 16; ++b) {
            int lanes = 0;
            for (uint32_t c = c0; c < std::min(c0 + 64, nch); ++c)
                if (16 * c + b < K) addr[lanes++] = pos[16 * c + b];
            cost += bank_cost(addr, lanes);
        }
    const uint32_t nb = uint32_t(ipow64(f.k, m - q));
    for (uint32_t a0 = 0; a0 < nb; a0 += 64)
        for (uint32_t rr = 0; rr < BS + 2; ++rr)
            for (uint32_t half = 0; half < 2; ++half) {
                int lanes = 0;
                for (uint32_t a = a0; a < std::min(a0 + 64, nb); ++a) {
                    int64_t X, Y;
                    lambda_levels(f, m - q, a, &X, &Y);
                    addr[lanes++] = (uint32_t((Y * BS) * W + X * BS) & ~3u) + rr * W + 4 * half;
                }
                cost += bank_cost(addr, lanes);
            }
    return cost;
}

bool build_tile_plan(const Fractal &f, uint32_t m, TilePlan *p, std::string *msg, uint32_t team) {
    *p = TilePlan();
    if (team != 256 && team != 64) {
        *msg = "team size must be 256 or 64";
        return false;
    }
    if (!tiled_supported(f)) {
        *msg = "the tiled step needs 2 <= s <= 4 and r >= 1";
        return false;
    }
    if (m < 1 || m > f.r) {
        *msg = "tile level must lie in [1, r]";
        return false;
    }
    uint64_t S = ipow64(f.s, m);
    if (S > 250 || box_alloc_bytes(uint32_t(S)) > 65535) {
        *msg = "tile level too large for 16-bit LDS offsets";
        return false;
    }
    const uint32_t q = block_level(f, m);
    // A team holds at most two 16-byte chunks, four halo cells and four
    // blocks per thread.
    const uint64_t K = ipow64(f.k, m);
    if (K + 30 > 2 * 16 * team || ipow64(f.k, m - q) > 4 * team) {
        *msg = team == 256 ? "tile level too large for one work-group" : "tile level too large for one wavefront";
        return false;
    }
    p->team = team;
    p->m = m;
    p->S = uint32_t(S);
    p->K = uint32_t(K);
    uint32_t cols;
    box_extent(f, m, &p->rows, &cols);
    // Box pitch: among the multiples of 4 in [cols, cols+64) whose box fits
    // the budget (or the smallest pitch when none fits, as for large
    // requested tile levels), those that keep the most work-groups resident
    // per CU by LDS, and among them the one with the fewest modelled bank
    // conflicts.
    p->W = (cols + 3) & ~3u;
    {
        const uint32_t least = p->rows * p->W + 8;
        auto resident = [&](uint32_t W) {
            const uint32_t per_team = ((p->rows * W + 8) + 15) & ~15u;
            return std::min(kMaxGroupsPerCU, kLdsPerCU / (per_team * (256 / team) + 256));
        };
        uint32_t most = resident(p->W);
        for (uint32_t W = p->W + 4; W < p->W + 64 && p->rows * W + 8 <= std::max(kBoxBudget, least); W += 4)
            most = std::max(most, resident(W));
        uint64_t best = ~uint64_t(0);
        const uint32_t W0 = p->W;
        for (uint32_t W = W0; W < W0 + 64; W += 4) {
            if (W > W0 && p->rows * W + 8 > std::max(kBoxBudget, least)) break;
            if (resident(W) < most) continue;
            const uint64_t c = box_pitch_cost(f, m, q, W);
            if (c < best) {
                best = c;
                p->W = W;
            }
        }
    }
    p->q = q;
    p->BS = uint32_t(ipow64(f.s, q));
    p->CB = uint32_t(ipow64(f.k, q));
    p->nblk = uint32_t(ipow64(f.k, m - q));
    p->box_bytes = p->rows * p->W + 8;
    p->lds_total = (p->box_bytes + 15) & ~15u;
    if (team == 64 && 4 * uint64_t(p->lds_total) > 65536) {
        *msg = "four wavefront boxes do not fit 64 KiB of LDS";
        return false;
    }
    p->rm = f.r - m;
    p->ntiles = ipow64(f.k, p->rm);
    p->Sc = uint32_t(ipow64(f.s, p->rm));
    p->lut0.resize(p->K);
    for (uint32_t i = 0; i < p->K; ++i) {
        int64_t x, y;
        lambda_levels(f, m, i, &x, &y);
        p->lut0[i] = uint16_t((y + 1) * p->W + (x + 1));
    }
    p->lut0_stride = (p->K + 16 + 15) & ~15u;  // >= every 16-entry read of any phase
    p->dummy = p->rows * p->W + 4;             // slack byte past every window read
    p->lut0p.assign(size_t(16) * p->lut0_stride, uint16_t(p->dummy));
    for (uint32_t ph = 0; ph < 16; ++ph)
        for (uint32_t i = 0; i < p->K; ++i) p->lut0p[size_t(ph) * p->lut0_stride + i + ph] = p->lut0[i];
    p->blk_pos.resize(p->K);
    {
        const uint32_t nq = (p->S + 3) / 4;
        p->blk_mask.assign(size_t(p->S) * nq, 0);
        for (uint32_t i = 0; i < p->K; ++i) {
            int64_t x, y;
            lambda_levels(f, m, i, &x, &y);
            p->blk_pos[i] = uint32_t(y * p->S + x);
            p->blk_mask[size_t(y) * nq + x / 4] |= 1u << (8 * (x % 4));
        }
    }
    p->lut1.resize(p->nblk);
    for (uint32_t b = 0; b < p->nblk; ++b) {
        int64_t X, Y;
        lambda_levels(f, m - q, b, &X, &Y);
        p->lut1[b] = uint16_t(Y * p->BS * p->W + X * p->BS);
    }
    std::memset(p->bid, 0xFF, sizeof(p->bid));
    p->brows = 0;
    for (uint32_t rr = 0; rr < p->BS; ++rr)
        for (uint32_t c = 0; c < p->BS; ++c) {
            int64_t v = nu_levels(f, q, c, rr);
            if (v >= 0) {
                p->bid[c + p->BS * rr] = uint8_t(v);
                p->brows = rr + 1;
            }
        }
    // Byte gathers from block rows to compact order: byte j of the block's
    // output is the cell with id j, at column c of row r; rows 0 and 1 feed
    // pack01 (row 0 as the low source, selectors 0-3, row 1 as the high one,
    // 4-7), rows 2 and 3 feed pack23 the same way; 12 selects a zero byte.
    for (uint32_t d = 0; d < 4; ++d) {
        uint32_t s01 = 0, s23 = 0;
        for (uint32_t b = 0; b < 4; ++b) {
            uint32_t a = 12, h = 12;
            const uint32_t j = 4 * d + b;
            for (uint32_t pos = 0; pos < p->BS * p->BS; ++pos)
                if (p->bid[pos] == j) {
                    const uint32_t c = pos % p->BS, r = pos / p->BS;
                    if (r < 2) a = r * 4 + c;
                    else h = (r - 2) * 4 + c;
                }
            s01 |= a << (8 * b);
            s23 |= h << (8 * b);
        }
        p->pack01[d] = s01;
        p->pack23[d] = s23;
    }
    const int64_t Si = p->S;
    uint32_t dir8 = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            for (uint32_t i = 0; i < p->K; ++i) {
                int64_t x, y;
                lambda_levels(f, m, i, &x, &y);
                int64_t tx = x + dx * Si, ty = y + dy * Si;
                if (tx < -1 || ty < -1 || tx > Si || ty > Si) continue;
                if (ty + 1 >= int64_t(p->rows) || tx + 1 >= int64_t(p->W)) continue;  // never read
                p->halo_src.push_back((dir8 << 29) | i);
                p->halo_dst.push_back(uint32_t((ty + 1) * p->W + (tx + 1)));
            }
            ++dir8;
        }
    if (p->halo_src.size() > 4 * team) {
        *msg = team == 256 ? "tile level too large for one work-group" : "tile level too large for one wavefront";
        return false;
    }
    // Neighbour tiles: the tiles' block corners are S * lambda_{r-m}(t); the
    // eight neighbours are nu_{r-m} of the neighbouring coarse coordinates
    // (section 3.1 at the coarse level), or none outside the fractal.
    if (p->ntiles * 8 > (uint64_t(1) << 28)) {
        *msg = "too many tiles for the neighbour table";
        return false;
    }
    p->nbr.resize(p->ntiles * 8);
    for (uint64_t t = 0; t < p->ntiles; ++t) {
        int64_t X, Y;
        lambda_levels(f, p->rm, t, &X, &Y);
        uint32_t d8 = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                int64_t v = nu_levels(f, p->rm, X + dx, Y + dy);
                p->nbr[t * 8 + d8++] = v < 0 ? 0xFFFFFFFFu : uint32_t(v);
            }
    }
    p->ok = true;
    return true;
}

bool build_edge_plan(const Fractal &f, uint32_t m, EdgePlan *p, std::string *msg) {
    *p = EdgePlan();
    if (!tiled_supported(f) || m < 1 || m > f.r) {
        *msg = "the edge form needs a tiled fractal and 1 <= m <= r";
        return false;
    }
    const uint32_t q = block_level(f, m);
    const uint32_t BS = uint32_t(ipow64(f.s, q)), CB = uint32_t(ipow64(f.k, q));
    const uint32_t G = uint32_t(ipow64(f.s, m - q));
    const uint64_t nb = ipow64(f.k, m - q), K = ipow64(f.k, m);
    // two source dwords for 3 x 3 blocks of up to 8 cells, else four
    const uint32_t nsrc = (BS == 3 && CB <= 8) ? 2 : 4, LW = 4 * nsrc;
    if (BS < 3 || CB > 16) {
        *msg = "the edge form needs blocks of side 3 or 4";
        return false;
    }
    if (K < 2 * LW) {
        *msg = "tile too small for the edge form";
        return false;
    }
    if (nb > 1024) {
        *msg = "more than 1024 blocks per tile";
        return false;
    }
    p->m = m;
    p->q = q;
    p->S = uint32_t(ipow64(f.s, m));
    p->K = uint32_t(K);
    p->BS = BS;
    p->CB = CB;
    p->G = G;
    p->nblk = uint32_t(nb);
    p->nsrc = nsrc;
    // block slots: block b of the tile sits at lambda_{m-q}(b) on the G x G grid
    const int64_t Gi = G;
    std::vector<int32_t> own(size_t(G + 2) * (G + 2), -1);  // (Y+1)*(G+2) + X+1 -> block
    auto at = [&](int64_t X, int64_t Y) -> int32_t & { return own[size_t(Y + 1) * (G + 2) + size_t(X + 1)]; };
    p->blk_xy.resize(2 * nb);
    for (uint64_t b = 0; b < nb; ++b) {
        int64_t X, Y;
        lambda_levels(f, m - q, b, &X, &Y);
        p->blk_xy[2 * b] = int32_t(X);
        p->blk_xy[2 * b + 1] = int32_t(Y);
        at(X, Y) = int32_t(b);
    }
    // halo items: blocks of the eight neighbour tiles that land on the ring
    // next to one of the tile's blocks; direction numbering as the neighbour
    // table (row-major over dy, dx in -1..1 without the centre)
    auto touches = [&](int64_t X, int64_t Y) {
        for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
                const int64_t x = X + dx, y = Y + dy;
                if (x >= 0 && y >= 0 && x < Gi && y < Gi && at(x, y) >= 0) return true;
            }
        return false;
    };
    std::vector<uint32_t> hd, hs;
    uint32_t dir8 = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            for (uint64_t b = 0; b < nb; ++b) {
                const int64_t X = p->blk_xy[2 * b] + dx * Gi, Y = p->blk_xy[2 * b + 1] + dy * Gi;
                if (X < -1 || Y < -1 || X > Gi || Y > Gi || !touches(X, Y)) continue;
                p->halo_xy.push_back(int32_t(X));
                p->halo_xy.push_back(int32_t(Y));
                hd.push_back((dir8 << 29) | uint32_t(b));
            }
            ++dir8;
        }
    p->nhalo = uint32_t(hd.size());
    if (p->nhalo > 512) {
        *msg = "more than 512 halo blocks per tile";
        return false;
    }
    // records: block b is record b, halo item h record nblk + h, and one
    // record of zeros (nrec - 1) stands for every position that holds no
    // block; the lanes of a wavefront write consecutive records
    const uint32_t zrec = p->nblk + p->nhalo;
    p->nrec = zrec + 1;
    p->rec_bytes = 16 * ((p->nrec + 3) & ~3u);
    std::vector<int32_t> ring(size_t(G + 2) * (G + 2), -1);  // halo item at (X, Y), X, Y in -1..G
    for (uint32_t h = 0; h < p->nhalo; ++h)
        ring[size_t(p->halo_xy[2 * h + 1] + 1) * (G + 2) + size_t(p->halo_xy[2 * h] + 1)] = int32_t(h);
    auto record_at = [&](int64_t X, int64_t Y) -> uint32_t {
        if (X < -1 || Y < -1 || X > Gi || Y > Gi) return zrec;
        const int32_t b = at(X, Y);
        if (b >= 0) return uint32_t(b);
        const int32_t h = ring[size_t(Y + 1) * (G + 2) + size_t(X + 1)];
        return h >= 0 ? p->nblk + uint32_t(h) : zrec;
    };
    p->blk.resize(4 * nb);
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t X = p->blk_xy[2 * b], Y = p->blk_xy[2 * b + 1];
        p->blk[4 * b] = record_at(X - 1, Y) | (record_at(X + 1, Y) << 16);
        p->blk[4 * b + 1] = record_at(X, Y - 1) | (record_at(X, Y + 1) << 16);
        p->blk[4 * b + 2] = record_at(X - 1, Y - 1) | (record_at(X + 1, Y - 1) << 16);
        p->blk[4 * b + 3] = record_at(X - 1, Y + 1) | (record_at(X + 1, Y + 1) << 16);
    }
    p->halo.resize(2 * size_t(p->nhalo));
    for (uint32_t h = 0; h < p->nhalo; ++h) {
        p->halo[2 * h] = hd[h];
        p->halo[2 * h + 1] = p->nblk + h;
    }
    // v_perm selectors: byte c of row r is cell bid(c, r) of the block's CB
    // bytes (dwords c0..c3), 12 (a zero byte) where the block has no cell
    uint8_t bid[16];
    std::memset(bid, 0xFF, sizeof(bid));
    for (uint32_t rr = 0; rr < BS; ++rr)
        for (uint32_t c = 0; c < BS; ++c) {
            const int64_t v = nu_levels(f, q, c, rr);
            if (v >= 0) bid[c + BS * rr] = uint8_t(v);
        }
    for (uint32_t rr = 0; rr < 4; ++rr) {
        uint32_t sa = 0, sb = 0;
        for (uint32_t c = 0; c < 4; ++c) {
            uint32_t a = 12, b = 12;
            const uint32_t j = (rr < BS && c < BS) ? bid[c + BS * rr] : 0xFFu;
            if (j != 0xFFu) {
                if (j < 8) a = j;
                else b = j - 8;
            }
            sa |= a << (8 * c);
            sb |= b << (8 * c);
        }
        p->unpack01[rr] = sa;
        p->unpack23[rr] = sb;
    }
    // compact dword d of the next states from rows (n0, n1) and (n2, n3)
    for (uint32_t d = 0; d < 4; ++d) {
        uint32_t s01 = 0, s23 = 0;
        for (uint32_t b = 0; b < 4; ++b) {
            uint32_t a = 12, h = 12;
            const uint32_t j = 4 * d + b;
            for (uint32_t pos = 0; pos < BS * BS; ++pos)
                if (bid[pos] == j) {
                    const uint32_t c = pos % BS, r = pos / BS;
                    if (r < 2) a = r * 4 + c;
                    else h = (r - 2) * 4 + c;
                }
            s01 |= a << (8 * b);
            s23 |= h << (8 * b);
        }
        p->pack01[d] = s01;
        p->pack23[d] = s23;
    }
    p->ok = true;
    return true;
}

void build_mfma_tables(const Fractal &f, MfmaTables *t) {
    *t = MfmaTables();
    const uint64_t K = uint64_t(f.r) * f.k;
    if (f.r == 0 || K > 192 || f.n > (uint64_t(1) << 28)) return;
    t->ktiles = uint32_t((K + 31) / 32);
    const uint32_t KB = 32 * t->ktiles;
    t->A.assign(size_t(16) * KB, 0);
    int64_t scale = 1;
    for (uint32_t mu = 0; mu < f.r; ++mu, scale *= f.s)
        for (uint32_t j = 0; j < f.k; ++j)
            for (uint32_t p = 0; p < 4; ++p) {
                t->A[p * KB + mu * f.k + j] = int8_t(((f.ox[j] * scale) >> (7 * p)) & 127);
                t->A[(4 + p) * KB + mu * f.k + j] = int8_t(((f.oy[j] * scale) >> (7 * p)) & 127);
            }
    // nu: row p = 7-bit plane p of j k^mu (five planes: indices < 2^32 <= 2^35)
    t->Anu.assign(size_t(16) * KB, 0);
    uint64_t kmu = 1;
    for (uint32_t mu = 0; mu < f.r; ++mu, kmu *= f.k)
        for (uint32_t j = 0; j < f.k; ++j)
            for (uint32_t p = 0; p < 5; ++p) t->Anu[p * KB + mu * f.k + j] = int8_t(((j * kmu) >> (7 * p)) & 127);
}

bool build_temporal_plan(const Fractal &f, uint32_t m, uint32_t h, uint32_t lds_limit, TemporalPlan *p,
                         std::string *msg) {
    *p = TemporalPlan();
    if (!tiled_supported(f) || m < 1 || m > f.r) {
        *msg = "temporal blocking needs a tiled fractal and 1 <= m <= r";
        return false;
    }
    const uint64_t S = ipow64(f.s, m), K = ipow64(f.k, m);
    if (h < 1 || h > S) {
        *msg = "the ring depth must lie in [1, tile side]";
        return false;
    }
    const uint64_t B = S + 2 * uint64_t(h), P = (B + 3) & ~uint64_t(3);
    const uint64_t box = (B * P + 15) & ~uint64_t(15);
    if (3 * box > lds_limit || K > (uint64_t(1) << 29)) {
        *msg = "the boxes of this tile level and ring depth exceed the LDS";
        return false;
    }
    p->m = m;
    p->S = uint32_t(S);
    p->K = uint32_t(K);
    p->h = h;
    p->B = uint32_t(B);
    p->P = uint32_t(P);
    p->box_bytes = uint32_t(box);
    p->lds = uint32_t(3 * box);
    const uint32_t rm = f.r - m;
    p->ntiles = ipow64(f.k, rm);
    if (p->ntiles * 8 > (uint64_t(1) << 28)) {
        *msg = "too many tiles for the neighbour table";
        return false;
    }
    p->self.resize(K);
    std::vector<int64_t> xs(K), ys(K);
    for (uint64_t j = 0; j < K; ++j) {
        lambda_levels(f, m, j, &xs[j], &ys[j]);
        p->self[j] = uint32_t((ys[j] + h) * P + (xs[j] + h));
    }
    // the cells of each neighbour tile inside the box; directions numbered
    // row by row, skipping the centre, as in the neighbour table
    const int64_t Si = int64_t(S), hi = h;
    uint32_t d8 = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            for (uint64_t j = 0; j < K; ++j) {
                const int64_t X = xs[j] + dx * Si + hi, Y = ys[j] + dy * Si + hi;
                if (X < 0 || Y < 0 || X >= int64_t(B) || Y >= int64_t(B)) continue;
                p->halo.push_back((d8 << 29) | uint32_t(j));
                p->halo.push_back(uint32_t(Y * int64_t(P) + X));
            }
            ++d8;
        }
    p->nbr.resize(p->ntiles * 8);
    for (uint64_t t = 0; t < p->ntiles; ++t) {
        int64_t X, Y;
        lambda_levels(f, rm, t, &X, &Y);
        uint32_t e = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const int64_t v = nu_levels(f, rm, X + dx, Y + dy);
                p->nbr[t * 8 + e++] = v < 0 ? 0xFFFFFFFFu : uint32_t(v);
            }
    }
    p->ok = true;
    return true;
}

uint64_t box_pitch(const Fractal &f) { return std::max<uint64_t>(16, (f.n + 15) & ~uint64_t(15)); }

void build_box_tables(const Fractal &f, BoxTables *b) {
    uint32_t L = 0;
    while (L + 1 <= f.r && ipow64(f.s, L + 1) <= 1024) ++L;
    b->L = L;
    b->SL = uint32_t(ipow64(f.s, L));
    b->LW = (b->SL + 31) / 32 + 1;
    b->NH = uint32_t(ipow64(f.s, f.r - L));
    b->low.assign(size_t(b->SL) * b->LW, 0);
    for (uint32_t y = 0; y < b->SL; ++y)
        for (uint32_t x = 0; x < b->SL; ++x)
            if (nu_levels(f, L, x, y) >= 0) b->low[size_t(y) * b->LW + x / 32] |= 1u << (x % 32);
    if (uint64_t(b->NH) * b->NH > (uint64_t(1) << 26)) {  // the box itself could not be allocated
        b->high.clear();
        return;
    }
    b->high.assign(size_t(b->NH) * b->NH, 0);
    for (uint32_t y = 0; y < b->NH; ++y)
        for (uint32_t x = 0; x < b->NH; ++x) b->high[size_t(y) * b->NH + x] = nu_levels(f, f.r - L, x, y) >= 0;
}

}  // namespace nbb
