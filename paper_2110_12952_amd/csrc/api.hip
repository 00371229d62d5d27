// C ABI of libnbbfrac (declared in include/nbbfrac.h): argument checks, the
// descriptor's device tables, and kernel launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/nbbfrac.h"
#include "edges_launch.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace nbb;

namespace {

thread_local std::string g_err;

nbb_status fail(nbb_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
nbb_status hip_fail(hipError_t e, const char *what) {
    return fail(NBB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// One device allocation holding a set of tables; offsets are 256-aligned.
struct DevBlob {
    void *ptr = nullptr;
    size_t bytes = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

struct nbb_fractal {
    Fractal f;
    MapTables maps;
    TilePlan tile;
    BoxTables box;
    MfmaTables mfma;
    uint32_t strategy = NBB_STRATEGY_DIRECT;
    // The tiled step runs in edge-record form (k_step_edges) when its plan
    // applies at the tile level and the strategy is TILED; otherwise (and for
    // TILED_BOX / TILED_WAVE) in byte-scatter form (k_step_tiled).
    EdgePlan edge;
    bool use_edges = false;
    DevBlob dedge;
    EdgeParams ep{};
    // Several generations per launch (NBB_STRATEGY_TEMPORAL): the plan and
    // its device tables; the tile plan above stays for batches.
    TemporalPlan temporal;
    DevBlob dtemp;
    TemporalParams tmp{};
    int device = 0;
    int cu_count = 256;
    DevBlob dmap, dtile, dbox, dmfma;
    MfmaLambda ml{};
    MapParams mp{};
    TileParams tp{};
    BoxParams bp{};
    uint32_t lam_words = 0, nu_halves = 0;
    // Plan of the LDS-resident batch step, made on a batch's first use:
    // 0 not tried yet, 1 built (res_tp, stepped res_teams tiles at a time),
    // 2 none (the state does not fit, or would take too many passes).
    mutable std::mutex res_mu;
    mutable int res_state = 0;
    mutable TileParams res_tp{};
    mutable uint32_t res_teams = 1;
    mutable DevBlob dres;
    // 32-phase scatter table of the bit-packed step, for the plan whose
    // (m, W, team) it records; rebuilt when the plan changes.
    mutable std::mutex pk_mu;
    mutable DevBlob dpk;
    mutable uint32_t pk_stride = 0, pk_m = 0, pk_W = 0, pk_team = 0;
};

struct nbb_plan {
    Fractal f;
    TilePlan tile;
    EdgePlan edge;
};

struct nbb_temporal_plan {
    Fractal f;
    TemporalPlan plan;
};

// A batch: groups of instances that share a tile plan, each stepped by one
// launch over the group's tiles, and instances stepped one by one.
struct BatchGroup {
    TileParams tp;           // the plan of the group's first descriptor; nbr / ntiles are the batch's
    bool edges = false;      // stepped in edge-record form (ep, with the batch's nbr / ntiles)
    EdgeParams ep{};
    uint32_t BS = 0, nsrc = 0;
    const uint32_t *rec = nullptr;
    std::vector<uint32_t> index;      // the group's instances (caller's numbering), in tile order
    std::vector<uint64_t> tiles_end;  // tiles of the first j+1 of them
};
struct BatchDirect {
    const nbb_fractal *f;
    uint64_t offset;
    uint32_t index;
};
// The small instances that run all their generations in LDS: one launch,
// one work-group each, every plan in one table.
struct ResidentSet {
    const TileParams *plans = nullptr;     // device table, one entry per plan
    const ResidentInstance *inst = nullptr;  // device table, in `index` order
    uint32_t *steps = nullptr;             // device: per-instance generation counts (nbb_batch_step_each)
    std::vector<uint32_t> index;           // the instances (caller's numbering)
    std::vector<uint32_t> passes;          // passes per generation of each
    uint32_t lds = 0;                      // LDS of the largest
};
// An instance is stepped in LDS only if a generation takes at most this many
// passes (each about a microsecond: a tile scatter, the rule, two barriers):
// beyond that the per-generation group launches are faster.
constexpr uint32_t kResidentMaxPasses = 8;
struct nbb_batch {
    int device = 0;
    int cu_count = 256;
    uint32_t count = 0;
    uint64_t cells = 0, tiles = 0, arena_bytes = 0;
    std::vector<BatchGroup> groups;
    ResidentSet resident;
    std::vector<BatchDirect> direct;
    DevBlob dtab;
    // with group or direct launches beside it, the resident launch runs on the
    // device's side stream, forked from and joined back to the caller's
    // stream, so that the two overlap
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // With several groups, group k > 0 runs on gstream[(k - 1) % size] (the
    // device's group streams, forked from the caller's stream and joined back
    // to it), so that one group's launches fill the start and the tail of
    // another's; empty when the batch has one group or was built without
    // allocation.
    std::vector<hipStream_t> gstream;
    std::vector<hipEvent_t> gjoin;  // one per group stream
    hipEvent_t gfork = nullptr;
};

namespace {

void blob_free(DevBlob *b) {
    if (b->ptr) (void)hipFree(b->ptr);
    b->ptr = nullptr;
    b->bytes = 0;
}

// Upload `parts` (host pointer, bytes) into one fresh device allocation and
// return the device address of each part.
nbb_status upload(DevBlob *blob, const void *const *src, const size_t *bytes, int nparts,
                  void **dst) {
    size_t total = 0;
    size_t off[8];
    for (int i = 0; i < nparts; ++i) {
        off[i] = total;
        total += align256(std::max<size_t>(bytes[i], 1));
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? fail(NBB_E_NOMEM, "device table allocation failed")
                                        : hip_fail(e, "hipMalloc");
    }
    for (int i = 0; i < nparts; ++i) {
        if (bytes[i]) {
            e = hipMemcpy(static_cast<char *>(p) + off[i], src[i], bytes[i], hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(p);
                return hip_fail(e, "hipMemcpy");
            }
        }
        dst[i] = static_cast<char *>(p) + off[i];
    }
    blob->ptr = p;
    blob->bytes = total;
    return NBB_OK;
}

nbb_status upload_maps(nbb_fractal *F) {
    const Fractal &f = F->f;
    const MapTables &t = F->maps;
    uint8_t ox[kMaxK], oy[kMaxK];
    for (uint32_t j = 0; j < f.k; ++j) {
        ox[j] = uint8_t(f.ox[j]);
        oy[j] = uint8_t(f.oy[j]);
    }
    const void *src[5] = {t.lam.data(), t.nu.data(), ox, oy, f.hl};
    size_t bytes[5] = {t.lam.size() * 4, t.nu.size() * 2, f.k, f.k, 256};
    void *dst[5];
    nbb_status s = upload(&F->dmap, src, bytes, 5, dst);
    if (s != NBB_OK) return s;
    MapParams &P = F->mp;
    P.k = f.k;
    P.s = f.s;
    P.r = f.r;
    P.n = uint32_t(f.n);
    P.cells_m1 = uint32_t(f.cells - 1);
    P.divk = make_udiv(f.k);
    P.divs = make_udiv(f.s);
    P.jl = t.jl;
    P.jl_top = t.jl_top;
    P.nchunks_l = t.nchunks_l;
    uint64_t kl = 1, sl = 1;
    for (uint32_t i = 0; i < t.jl; ++i) {
        kl *= f.k;
        sl *= f.s;
    }
    P.kl = uint32_t(kl);
    P.sl = uint32_t(sl);
    P.divkl = make_udiv(P.kl);
    P.lam_top_off = t.lam_top_off;
    P.jn = t.jn;
    P.jn_top = t.jn_top;
    P.nchunks_n = t.nchunks_n;
    uint64_t sn = 1, kn = 1, st = 1;
    for (uint32_t i = 0; i < t.jn; ++i) {
        sn *= f.s;
        kn *= f.k;
    }
    for (uint32_t i = 0; i < t.jn_top; ++i) st *= f.s;
    P.sn = uint32_t(sn);
    P.kn = uint32_t(kn);
    P.sn_top = uint32_t(st);
    P.divsn = make_udiv(P.sn);
    P.nu_top_off = t.nu_top_off;
    P.lam_lut = static_cast<const uint32_t *>(dst[0]);
    P.nu_lut = static_cast<const uint16_t *>(dst[1]);
    P.ox = static_cast<const uint8_t *>(dst[2]);
    P.oy = static_cast<const uint8_t *>(dst[3]);
    P.hl = static_cast<const uint8_t *>(dst[4]);
    F->lam_words = uint32_t(t.lam.size());
    F->nu_halves = uint32_t(t.nu.size());
    return NBB_OK;
}

nbb_status upload_tile(nbb_fractal *F, const TilePlan &p, DevBlob *blob, TileParams *T) {
    const void *src[7] = {p.lut0p.data(), p.lut1.data(), p.halo_src.data(), p.halo_dst.data(), p.nbr.data(),
                          p.blk_pos.data(), p.blk_mask.data()};
    size_t bytes[7] = {p.lut0p.size() * 2, p.lut1.size() * 2, p.halo_src.size() * 4, p.halo_dst.size() * 4,
                       p.nbr.size() * 4, p.blk_pos.size() * 4, p.blk_mask.size() * 4};
    void *dst[7];
    nbb_status s = upload(blob, src, bytes, 7, dst);
    if (s != NBB_OK) return s;
    *T = TileParams{};
    T->team = p.team;
    T->m = p.m;
    T->S = p.S;
    T->K = p.K;
    T->W = p.W;
    T->q = p.q;
    T->BS = p.BS;
    T->CB = p.CB;
    T->nblk = p.nblk;
    T->brows = p.brows;
    T->box_bytes = p.box_bytes;
    T->lds_total = p.lds_total;
    T->rm = p.rm;
    T->ntiles = uint32_t(p.ntiles);
    T->Sc = p.Sc;
    T->halo_count = uint32_t(p.halo_src.size());
    T->cells = uint32_t(F->f.cells);
    T->lut0_stride = p.lut0_stride;
    T->dummy = p.dummy;
    T->lut0p = static_cast<const uint16_t *>(dst[0]);
    T->lut1 = static_cast<const uint16_t *>(dst[1]);
    T->halo_src = static_cast<const uint32_t *>(dst[2]);
    T->halo_dst = static_cast<const uint32_t *>(dst[3]);
    T->nbr = static_cast<const uint32_t *>(dst[4]);
    T->blk_pos = static_cast<const uint32_t *>(dst[5]);
    T->blk_mask = static_cast<const uint32_t *>(dst[6]);
    T->divK = make_udiv(p.K);
    T->divS = make_udiv(p.S);
    std::memcpy(T->pack01, p.pack01, sizeof(T->pack01));
    std::memcpy(T->pack23, p.pack23, sizeof(T->pack23));
    return NBB_OK;
}

// Uploads the temporal plan's tables (cell positions, ring items, neighbour
// tiles) into one allocation.
nbb_status upload_temporal(const TemporalPlan &p, DevBlob *blob, TemporalParams *T) {
    const void *src[3] = {p.self.data(), p.halo.data(), p.nbr.data()};
    size_t bytes[3] = {p.self.size() * 4, p.halo.size() * 4, p.nbr.size() * 4};
    void *dst[3];
    nbb_status s = upload(blob, src, bytes, 3, dst);
    if (s != NBB_OK) return s;
    *T = TemporalParams{};
    T->K = p.K;
    T->B = p.B;
    T->P = p.P;
    T->h = p.h;
    T->box_bytes = p.box_bytes;
    T->nhalo = uint32_t(p.halo.size() / 2);
    T->ntiles = uint32_t(p.ntiles);
    T->self = static_cast<const uint32_t *>(dst[0]);
    T->halo = static_cast<const uint32_t *>(dst[1]);
    T->nbr = static_cast<const uint32_t *>(dst[2]);
    return NBB_OK;
}

// Uploads the edge plan's tables; the neighbour table is the tile plan's
// (same level), already on the device at T.nbr.
nbb_status upload_edges(const EdgePlan &p, const TileParams &T, DevBlob *blob, EdgeParams *E) {
    const void *src[2] = {p.blk.data(), p.halo.data()};
    size_t bytes[2] = {p.blk.size() * 4, p.halo.size() * 4};
    void *dst[2];
    nbb_status s = upload(blob, src, bytes, 2, dst);
    if (s != NBB_OK) return s;
    *E = EdgeParams{};
    E->K = p.K;
    E->CB = p.CB;
    E->nblk = p.nblk;
    E->nhalo = p.nhalo;
    E->ntiles = T.ntiles;
    E->rec_bytes = p.rec_bytes;
    std::memcpy(E->unpack01, p.unpack01, sizeof(E->unpack01));
    std::memcpy(E->unpack23, p.unpack23, sizeof(E->unpack23));
    std::memcpy(E->pack01, p.pack01, sizeof(E->pack01));
    std::memcpy(E->pack23, p.pack23, sizeof(E->pack23));
    E->blk = static_cast<const uint32_t *>(dst[0]);
    E->halo = static_cast<const uint32_t *>(dst[1]);
    E->nbr = T.nbr;
    return NBB_OK;
}

// Builds and uploads the edge plan at the tile plan's level for a TILED
// descriptor; leaves the byte-scatter form in place where it does not apply.
// The edge form gives each thread whole blocks, one per pass of the
// work-group; where the blocks fill less than three quarters of the passes'
// thread slots the byte-scatter form measured faster (H r10 at level 4, 343
// blocks over two passes of 256 threads: 180 us per generation against 168;
// triangle r16, 243 blocks in one pass: 26.3 against 28.5; carpet r9, 512
// blocks in two: 60.8 against 65.2).  `force`: take the edge form wherever
// its plan applies.
nbb_status setup_edges(nbb_fractal *F, bool force = false) {
    blob_free(&F->dedge);
    F->use_edges = false;
    F->edge = EdgePlan();
    if (F->strategy != NBB_STRATEGY_TILED || F->tile.team != 256) return NBB_OK;
    std::string msg;
    EdgePlan p;
    if (!build_edge_plan(F->f, F->tile.m, &p, &msg)) return NBB_OK;
    const uint32_t passes = (p.nblk + 255) / 256;
    if (!force && 4 * p.nblk < 3 * 256 * passes) return NBB_OK;
    nbb_status st = upload_edges(p, F->tp, &F->dedge, &F->ep);
    if (st != NBB_OK) return st;
    F->edge = std::move(p);
    F->use_edges = true;
    return NBB_OK;
}

nbb_status upload_mfma(nbb_fractal *F) {
    if (!F->mfma.ktiles) return NBB_OK;
    const void *src[2] = {F->mfma.A.data(), F->mfma.Anu.data()};
    size_t bytes[2] = {F->mfma.A.size(), F->mfma.Anu.size()};
    void *dst[2];
    nbb_status s = upload(&F->dmfma, src, bytes, 2, dst);
    if (s != NBB_OK) return s;
    F->ml.ktiles = F->mfma.ktiles;
    F->ml.A = static_cast<const int8_t *>(dst[0]);
    F->ml.Anu = static_cast<const int8_t *>(dst[1]);
    return NBB_OK;
}

nbb_status upload_box(nbb_fractal *F) {
    const BoxTables &b = F->box;
    if (b.high.empty()) return NBB_OK;  // box too large to exist; box calls report NBB_E_RANGE
    const void *src[2] = {b.low.data(), b.high.data()};
    size_t bytes[2] = {b.low.size() * 4, b.high.size()};
    void *dst[2];
    nbb_status s = upload(&F->dbox, src, bytes, 2, dst);
    if (s != NBB_OK) return s;
    BoxParams &B = F->bp;
    B.n = uint32_t(F->f.n);
    B.SL = b.SL;
    B.LW = b.LW;
    B.NH = b.NH;
    B.divSL = make_udiv(b.SL);
    B.low = static_cast<const uint32_t *>(dst[0]);
    B.high = static_cast<const uint8_t *>(dst[1]);
    B.pitch = box_pitch(F->f);
    // Rows per work-group: enough work-groups to fill the chip, long enough
    // bands that the two extra rows each band reads stay a small fraction.
    const uint64_t gx = (B.pitch / 16 + 255) / 256;
    uint32_t rows = 64;
    while (rows > 8 && gx * ((F->f.n + rows - 1) / rows) < uint64_t(F->cu_count) * 16) rows /= 2;
    B.rows_per_wg = rows;
    return NBB_OK;
}

nbb_status check_device(const nbb_fractal *f) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != f->device) return fail(NBB_E_INVALID, "descriptor belongs to another device");
    return NBB_OK;
}

bool overlap(const void *a, const void *b, uint64_t len) {
    uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + len && y < x + len;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

const uint32_t kRuleMask = 0x1FFu | (0x1FFu << 16) | (1u << 31);

int map_grid(const nbb_fractal *F, uint64_t work_items) {
    uint64_t g = (work_items + 511) / 512;
    uint64_t cap = uint64_t(F->cu_count) * 4;
    return int(std::max<uint64_t>(1, std::min(g, cap)));
}

nbb_status launched(hipError_t e, const char *what) {
    if (e != hipSuccess) return hip_fail(e, what);
    return NBB_OK;
}

nbb_status check_box_args(const nbb_fractal *f, const void *p, uint64_t pitch, uint64_t len) {
    if (f->box.high.empty() || !f->dbox.ptr) return fail(NBB_E_RANGE, "the box of this fractal is too large");
    if (!p) return fail(NBB_E_INVALID, "null state pointer");
    if (!aligned16(p)) return fail(NBB_E_INVALID, "box state must be 16-byte aligned");
    if (pitch < f->f.n || pitch % 16 != 0)
        return fail(NBB_E_INVALID, "pitch must be >= n and a multiple of 16");
    if (pitch > 0xFFFFFFFFull) return fail(NBB_E_RANGE, "pitch too large");
    if (len != f->f.n * pitch) return fail(NBB_E_INVALID, "len must equal n * pitch");
    return NBB_OK;
}

}  // namespace

extern "C" {

const char *nbb_last_error(void) { return g_err.c_str(); }

const char *nbb_status_string(nbb_status s) {
    switch (s) {
        case NBB_OK: return "NBB_OK";
        case NBB_E_INVALID: return "NBB_E_INVALID";
        case NBB_E_RANGE: return "NBB_E_RANGE";
        case NBB_E_NOMEM: return "NBB_E_NOMEM";
        case NBB_E_DEVICE: return "NBB_E_DEVICE";
    }
    return "unknown";
}

nbb_status nbb_plan_build(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r,
                          uint32_t tile_level, nbb_plan **out, nbb_plan_view *view) {
    if (!out || !view) return fail(NBB_E_INVALID, "out and view must not be NULL");
    *out = nullptr;
    nbb_plan *p = new (std::nothrow) nbb_plan;
    if (!p) return fail(NBB_E_NOMEM, "host allocation failed");
    std::string msg;
    int v = validate_fractal(k, s, offsets, r, &p->f, &msg);
    if (v) {
        delete p;
        return fail(v == 2 ? NBB_E_RANGE : NBB_E_INVALID, msg);
    }
    uint32_t m = tile_level ? tile_level : auto_tile_level(p->f);
    if (!build_tile_plan(p->f, m, &p->tile, &msg)) {
        delete p;
        return fail(NBB_E_INVALID, msg);
    }
    const TilePlan &t = p->tile;
    view->tile_level = t.m;
    view->tile_side = t.S;
    view->tile_cells = t.K;
    view->block_level = t.q;
    view->block_side = t.BS;
    view->blocks = t.nblk;
    view->halo_count = uint32_t(t.halo_src.size());
    view->box_pitch = t.W;
    view->box_rows = t.rows;
    view->lds_bytes = t.lds_total;
    view->tiles = t.ntiles;
    view->lut0 = t.lut0.data();
    view->lut1 = t.lut1.data();
    view->halo_src = t.halo_src.data();
    view->halo_dst = t.halo_dst.data();
    view->nbr = t.nbr.data();
    view->edge_ok = build_edge_plan(p->f, t.m, &p->edge, &msg) ? 1u : 0u;
    const EdgePlan &e = p->edge;
    view->edge_grid = e.G;
    view->edge_records = e.nrec;
    view->edge_rec_bytes = e.rec_bytes;
    view->edge_halo_count = e.nhalo;
    view->edge_nsrc = e.nsrc;
    for (int i = 0; i < 4; ++i) {
        view->edge_unpack[i] = e.unpack01[i];
        view->edge_unpack[4 + i] = e.unpack23[i];
        view->edge_pack[i] = e.pack01[i];
        view->edge_pack[4 + i] = e.pack23[i];
    }
    view->edge_blk = e.blk.data();
    view->edge_halo = e.halo.data();
    *out = p;
    return NBB_OK;
}

void nbb_plan_free(nbb_plan *p) { delete p; }

nbb_status nbb_temporal_plan_build(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r, uint32_t tile_level,
                                   uint32_t depth, uint32_t lds_limit, nbb_temporal_plan **out,
                                   nbb_temporal_view *view) {
    if (!out || !view) return fail(NBB_E_INVALID, "null argument");
    *out = nullptr;
    auto *p = new (std::nothrow) nbb_temporal_plan;
    if (!p) return fail(NBB_E_NOMEM, "host allocation failed");
    std::string msg;
    int v = validate_fractal(k, s, offsets, r, &p->f, &msg);
    if (v) {
        delete p;
        return fail(v == 2 ? NBB_E_RANGE : NBB_E_INVALID, msg);
    }
    if (!build_temporal_plan(p->f, tile_level, depth, lds_limit ? lds_limit : 163840u, &p->plan, &msg)) {
        delete p;
        return fail(NBB_E_INVALID, msg);
    }
    const TemporalPlan &t = p->plan;
    std::memset(view, 0, sizeof(*view));
    view->tile_level = t.m;
    view->tile_side = t.S;
    view->tile_cells = t.K;
    view->depth = t.h;
    view->box_side = t.B;
    view->box_pitch = t.P;
    view->lds_bytes = t.lds;
    view->halo_count = uint32_t(t.halo.size() / 2);
    view->tiles = t.ntiles;
    view->self = t.self.data();
    view->halo = t.halo.data();
    view->nbr = t.nbr.data();
    *out = p;
    return NBB_OK;
}

void nbb_temporal_plan_free(nbb_temporal_plan *p) { delete p; }

nbb_status nbb_create(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r, nbb_fractal **out) {
    if (!out) return fail(NBB_E_INVALID, "out is NULL");
    *out = nullptr;
    nbb_fractal *F = new (std::nothrow) nbb_fractal;
    if (!F) return fail(NBB_E_NOMEM, "host allocation failed");
    std::string msg;
    int v = validate_fractal(k, s, offsets, r, &F->f, &msg);
    if (v) {
        delete F;
        return fail(v == 2 ? NBB_E_RANGE : NBB_E_INVALID, msg);
    }
    hipError_t e = hipGetDevice(&F->device);
    if (e != hipSuccess) {
        delete F;
        (void)hipGetLastError();
        return hip_fail(e, "hipGetDevice");
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, F->device) == hipSuccess && cus > 0)
        F->cu_count = cus;
    build_map_tables(F->f, &F->maps);
    build_box_tables(F->f, &F->box);
    build_mfma_tables(F->f, &F->mfma);
    nbb_status st = upload_maps(F);
    if (st == NBB_OK) st = upload_box(F);
    if (st == NBB_OK) st = upload_mfma(F);
    if (st == NBB_OK) {
        if (tiled_supported(F->f)) {
            if (build_tile_plan(F->f, auto_tile_level(F->f), &F->tile, &msg)) {
                st = upload_tile(F, F->tile, &F->dtile, &F->tp);
                if (st == NBB_OK) F->strategy = NBB_STRATEGY_TILED;
                if (st == NBB_OK) st = setup_edges(F);
            }
        }
    }
    if (st != NBB_OK) {
        blob_free(&F->dmap);
        blob_free(&F->dbox);
        blob_free(&F->dtile);
        blob_free(&F->dedge);
        blob_free(&F->dmfma);
        delete F;
        return st;
    }
    *out = F;
    return NBB_OK;
}

void nbb_destroy(nbb_fractal *F) {
    if (!F) return;
    blob_free(&F->dres);
    blob_free(&F->dpk);
    blob_free(&F->dtemp);
    blob_free(&F->dmap);
    blob_free(&F->dbox);
    blob_free(&F->dtile);
    blob_free(&F->dedge);
    blob_free(&F->dmfma);
    delete F;
}

nbb_status nbb_query(const nbb_fractal *F, nbb_info *info) {
    if (!F || !info) return fail(NBB_E_INVALID, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n = F->f.n;
    info->cells = F->f.cells;
    info->k = F->f.k;
    info->s = F->f.s;
    info->r = F->f.r;
    info->strategy = F->strategy;
    if (F->strategy != NBB_STRATEGY_DIRECT) {
        info->tiles = F->tile.ntiles;
        info->tile_level = F->tile.m;
        info->tile_side = F->tile.S;
        info->halo_cells = uint32_t(F->tile.halo_src.size());
        info->lds_bytes = F->tile.lds_total;
    } else {
        info->tiles = F->f.cells;
        info->tile_level = 0;
        info->tile_side = 1;
    }
    info->bbox_pitch = box_pitch(F->f);
    info->device_table_bytes = F->dmap.bytes + F->dbox.bytes + F->dtile.bytes + F->dedge.bytes + F->dmfma.bytes;
    uint32_t ebpt = 0, ehpt = 0;
    if (F->use_edges && edge_case(F->edge.nblk, F->edge.nhalo, &ebpt, &ehpt)) info->lds_bytes = edge_lds_bytes(ebpt, ehpt);
    info->tiled_form = F->strategy == NBB_STRATEGY_DIRECT ? 0u : (F->use_edges ? 1u : 2u);
    info->box_low_side = F->box.SL;
    info->box_high_side = F->box.high.empty() ? 0 : F->box.NH;
    if (F->strategy == NBB_STRATEGY_TEMPORAL) {
        const TemporalPlan &t = F->temporal;
        info->tiles = t.ntiles;
        info->tile_level = t.m;
        info->tile_side = t.S;
        info->halo_cells = uint32_t(t.halo.size() / 2);
        info->lds_bytes = t.lds;
        info->tiled_form = 3;
        info->temporal_depth = t.h;
    }
    info->device_table_bytes += F->dtemp.bytes;
    return NBB_OK;
}

nbb_status nbb_configure(nbb_fractal *F, uint32_t strategy, uint32_t tile_level) {
    if (!F) return fail(NBB_E_INVALID, "null descriptor");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    if (strategy == NBB_STRATEGY_TEMPORAL) return nbb_configure_temporal(F, tile_level, 0);
    if (strategy == NBB_STRATEGY_AUTO) strategy = tiled_supported(F->f) ? NBB_STRATEGY_TILED : NBB_STRATEGY_DIRECT;
    if (strategy == NBB_STRATEGY_DIRECT) {
        if (tile_level != 0) return fail(NBB_E_INVALID, "the direct strategy takes no tile level");
        F->strategy = NBB_STRATEGY_DIRECT;
        blob_free(&F->dtemp);
        F->temporal = TemporalPlan();
        blob_free(&F->dedge);
        F->use_edges = false;
        return NBB_OK;
    }
    if (strategy != NBB_STRATEGY_TILED && strategy != NBB_STRATEGY_TILED_WAVE &&
        strategy != NBB_STRATEGY_TILED_BOX && strategy != NBB_STRATEGY_TILED_EDGE)
        return fail(NBB_E_INVALID, "unknown strategy");
    const uint32_t team = strategy == NBB_STRATEGY_TILED_WAVE ? 64u : 256u;
    std::string msg;
    TilePlan plan;
    uint32_t m = tile_level ? tile_level : auto_tile_level(F->f);
    if (!tiled_supported(F->f) || !build_tile_plan(F->f, m, &plan, &msg, team))
        return fail(NBB_E_INVALID, msg.empty() ? "the tiled step does not support this fractal" : msg);
    if (strategy == NBB_STRATEGY_TILED_EDGE) {
        EdgePlan probe;
        if (!build_edge_plan(F->f, m, &probe, &msg))
            return fail(NBB_E_INVALID, "the edge-record form does not apply: " + msg);
    }
    DevBlob blob;
    TileParams T;
    st = upload_tile(F, plan, &blob, &T);
    if (st != NBB_OK) return st;
    blob_free(&F->dtile);
    F->dtile = blob;
    F->tile = std::move(plan);
    F->tp = T;
    F->strategy = (strategy == NBB_STRATEGY_TILED_BOX || strategy == NBB_STRATEGY_TILED_EDGE) ? NBB_STRATEGY_TILED
                                                                                                 : strategy;
    blob_free(&F->dtemp);
    F->temporal = TemporalPlan();
    if (strategy == NBB_STRATEGY_TILED_BOX) {
        blob_free(&F->dedge);
        F->use_edges = false;
        F->edge = EdgePlan();
        return NBB_OK;
    }
    return setup_edges(F, strategy == NBB_STRATEGY_TILED_EDGE);
}

// Most LDS one work-group may take on the current device.
static uint32_t device_lds_per_group();

// Automatic temporal plan: over the tile levels of side S <= 81 with ring
// depth h = min(16, S), the one with the least estimated time per generation
//   (3 + w) / h + 1e-4 (S + 2h)^2 w  microseconds,  w = max(tiles, CUs) / CUs:
// a launch (about 3 us) and each wave of tiles over the CUs (about 1 us of
// loads, stores and scheduling) per h generations, plus the box's cells per
// generation.  Fitted to measurements (256 CUs, per generation, B3/S23):
// the triangle r = 10 takes 3.7 us per generation in the tiled step and
// 1.18 / 1.14 / 1.73 / 3.6 us at levels 4 / 5 / 6 / 7 with h = 16, 2.19 /
// 1.43 / 1.19 / 1.14 / 1.32 us at level 5 with h = 2 / 4 / 8 / 16 / 32; over
// triangles r 8-13, carpets and H fractals r 4-7 and chandeliers r 6-9 the
// estimate picks the measured best level in 14 of 18 cases (the others are
// within 25 % of it).
static void auto_temporal(const Fractal &f, uint32_t cu_count, uint32_t *m, uint32_t *h) {
    const double cus = double(std::max(cu_count, 1u));
    double best_t = -1.0;
    uint32_t best_m = 1;
    uint64_t S = 1;
    for (uint32_t lv = 1; lv <= f.r; ++lv) {
        S *= f.s;
        if (lv > 1 && S > 81) break;
        if (*m && lv != *m) continue;
        const double hh = double(*h ? *h : std::min<uint64_t>(16, S));
        double tiles = 1.0;
        for (uint32_t i = lv; i < f.r; ++i) tiles *= f.k;
        const double w = std::max(tiles, cus) / cus, B = double(S) + 2.0 * hh;
        const double t = (3.0 + w) / hh + 1e-4 * B * B * w;
        if (best_t < 0.0 || t < best_t) {
            best_t = t;
            best_m = lv;
        }
    }
    if (!*m) *m = best_m;
    if (!*h) {
        uint64_t side = 1;
        for (uint32_t i = 0; i < *m; ++i) side *= f.s;
        *h = uint32_t(std::min<uint64_t>(16, side));
    }
}

nbb_status nbb_configure_temporal(nbb_fractal *F, uint32_t tile_level, uint32_t depth) {
    if (!F) return fail(NBB_E_INVALID, "null descriptor");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    if (!tiled_supported(F->f)) return fail(NBB_E_INVALID, "temporal blocking needs 2 <= s <= 4 and r >= 1");
    if (tile_level > F->f.r) return fail(NBB_E_INVALID, "tile level must lie in [1, r]");
    uint32_t m = tile_level, h = depth;
    auto_temporal(F->f, uint32_t(F->cu_count), &m, &h);
    std::string msg;
    TemporalPlan plan;
    if (!build_temporal_plan(F->f, m, h, device_lds_per_group(), &plan, &msg)) return fail(NBB_E_INVALID, msg);
    DevBlob blob;
    TemporalParams T;
    st = upload_temporal(plan, &blob, &T);
    if (st != NBB_OK) return st;
    blob_free(&F->dtemp);
    F->dtemp = blob;
    F->temporal = std::move(plan);
    F->tmp = T;
    F->strategy = NBB_STRATEGY_TEMPORAL;
    return NBB_OK;
}

nbb_status nbb_autotune(nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps, uint32_t rule,
                        void *stream, nbb_info *info) {
    if (!F || !a || !b) return fail(NBB_E_INVALID, "null argument");
    if (steps == 0) return fail(NBB_E_INVALID, "steps must be >= 1");
    if (len != F->f.cells) return fail(NBB_E_INVALID, "len must equal k^r");
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "state buffers must be 16-byte aligned");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    // Candidates: (strategy, level, ring depth).  Tile levels whose plan
    // fits a work-group, keeping those with >= 128 cells per tile and the
    // largest; several generations per launch at the automatic plan and at
    // each level of side <= 81 with depths 8 and 16 (when steps allows more
    // than one generation per launch).
    struct Cand {
        uint32_t strategy, level, depth;
    };
    std::vector<Cand> cand;
    if (tiled_supported(F->f)) {
        std::vector<uint32_t> fit;
        for (uint32_t m = 1; m <= F->f.r; ++m) {
            uint64_t K = 1, S = 1;
            for (uint32_t i = 0; i < m; ++i) {
                K *= F->f.k;
                S *= F->f.s;
            }
            if (K + 30 > 2 * 16 * 256 || S > 250) break;
            fit.push_back(m);
        }
        for (size_t i = 0; i < fit.size(); ++i) {
            uint64_t K = 1;
            for (uint32_t j = 0; j < fit[i]; ++j) K *= F->f.k;
            if (K >= 128 || i + 1 == fit.size()) {
                cand.push_back({NBB_STRATEGY_TILED_EDGE, fit[i], 0});  // edge records (skipped where they do not apply)
                cand.push_back({NBB_STRATEGY_TILED_BOX, fit[i], 0});   // byte scatter
                cand.push_back({NBB_STRATEGY_TILED_WAVE, fit[i], 0});  // skipped where it does not fit
            }
        }
        if (steps > 1) {
            cand.push_back({NBB_STRATEGY_TEMPORAL, 0, 0});
            uint64_t S = 1;
            for (uint32_t m = 1; m <= F->f.r; ++m) {
                S *= F->f.s;
                if (S > 81) break;
                for (uint32_t h : {8u, 16u})
                    if (h <= S) cand.push_back({NBB_STRATEGY_TEMPORAL, m, h});
            }
        }
    }
    cand.push_back({NBB_STRATEGY_DIRECT, 0, 0});
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    float best_ms = -1.0f;
    Cand best{0, 0, 0};
    auto apply = [&](const Cand &c) {
        return c.strategy == NBB_STRATEGY_TEMPORAL ? nbb_configure_temporal(F, c.level, c.depth)
                                                   : nbb_configure(F, c.strategy, c.level);
    };
    for (const auto &c : cand) {
        if (apply(c) != NBB_OK) continue;  // plan does not fit: skip it
        st = nbb_step_compact(F, a, b, len, 1, rule, nullptr, stream);
        if (st == NBB_OK && (e = hipEventRecord(e0, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
        if (st == NBB_OK) st = nbb_step_compact(F, b, a, len, steps, rule, nullptr, stream);
        if (st == NBB_OK && (e = hipEventRecord(e1, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
        if (st == NBB_OK && (e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
        float ms = 0.0f;
        if (st == NBB_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
        if (st != NBB_OK) break;
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != NBB_OK) return st;
    if (best_ms < 0.0f) return fail(NBB_E_INVALID, "no strategy could be configured");
    st = apply(best);
    if (st == NBB_OK && info) st = nbb_query(F, info);
    return st;
}

nbb_status nbb_batch_create(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                            void *stream, nbb_batch **out) {
    return nbb_batch_create_ex(fractals, offsets, count, 0, stream, out);
}

static uint32_t device_lds_per_group() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
        (void)hipGetLastError();
        return 65536;
    }
    return uint32_t(std::min(v, 163840));
}

// The LDS-resident plan of F, built on first use and kept with F: the tile
// level and tiles per pass with the fewest passes per generation (ties: the
// larger level) among those whose boxes, two state copies and neighbour table
// fit one work-group's LDS.  NULL if none does in kResidentMaxPasses passes.
static const TileParams *resident_plan(const nbb_fractal *F, uint32_t *teams) {
    std::lock_guard<std::mutex> lock(F->res_mu);
    if (F->res_state == 0) {
        F->res_state = 2;
        const uint32_t budget = device_lds_per_group();
        if (tiled_supported(F->f) && 2 * F->f.cells < budget) {
            TilePlan best;
            uint32_t best_passes = kResidentMaxPasses + 1, best_teams = 1;
            for (uint32_t m = F->f.r; m >= 1; --m) {
                TilePlan plan;
                std::string msg;
                if (!build_tile_plan(F->f, m, &plan, &msg, 256)) continue;
                if (uint64_t(plan.ntiles) * plan.K != F->f.cells) continue;
                TileParams probe{};
                probe.K = plan.K;
                probe.lds_total = plan.lds_total;
                probe.halo_count = uint32_t(plan.halo_src.size());
                probe.nblk = plan.nblk;
                const uint32_t nt = uint32_t(plan.ntiles);
                for (uint32_t t : {4u, 2u, 1u}) {
                    if (t > nt && t > 1) continue;
                    if (!resident_fits(probe, t) || resident_lds_bytes(probe, nt, t) > budget) continue;
                    const uint32_t passes = (nt + t - 1) / t;
                    if (passes < best_passes) {
                        best = plan;
                        best_passes = passes;
                        best_teams = t;
                    }
                    break;  // more tiles per pass is never worse
                }
            }
            if (best_passes <= kResidentMaxPasses &&
                upload_tile(const_cast<nbb_fractal *>(F), best, &F->dres, &F->res_tp) == NBB_OK) {
                F->res_teams = best_teams;
                F->res_state = 1;
            }
        }
    }
    if (F->res_state != 1) return nullptr;
    *teams = F->res_teams;
    return &F->res_tp;
}

// The device's streams beside the caller's (created on first use, kept
// until the process ends; default priority, non-blocking): slot 0 for
// resident launches, slots 1 .. kGroupStreams for the groups of a batch.
constexpr int kGroupStreams = 3;
static hipError_t device_stream(int dev, int slot, hipStream_t *out) {
    static std::mutex mu;
    static std::vector<std::vector<hipStream_t>> pool;
    std::lock_guard<std::mutex> lock(mu);
    if (pool.size() <= size_t(dev)) pool.resize(dev + 1);
    std::vector<hipStream_t> &p = pool[dev];
    if (p.empty()) p.assign(1 + kGroupStreams, nullptr);
    if (!p[slot]) {
        hipError_t e = hipStreamCreateWithFlags(&p[slot], hipStreamNonBlocking);
        if (e != hipSuccess) {
            p[slot] = nullptr;
            return e;
        }
    }
    *out = p[slot];
    return hipSuccess;
}
static hipError_t resident_stream(int dev, hipStream_t *out) { return device_stream(dev, 0, out); }

static void batch_free(nbb_batch *B) {
    if (B->fork) (void)hipEventDestroy(B->fork);
    if (B->join) (void)hipEventDestroy(B->join);
    if (B->gfork) (void)hipEventDestroy(B->gfork);
    for (hipEvent_t ev : B->gjoin) (void)hipEventDestroy(ev);
    blob_free(&B->dtab);
    delete B;
}

// Builds a batch.  Its device tables go to one fresh allocation, or, when
// `fixed` is given, to those `fixed_cap` bytes (no allocation: the instance
// tables are written by kernels whose arguments carry them, nothing waits on
// the stream, and no instance is stepped in LDS, since those plans are built
// on the device on first use).
static nbb_status batch_create(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                               uint32_t flags, void *stream, uint8_t *fixed, size_t fixed_cap, nbb_batch **out) {
    if (!out) return fail(NBB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (count && (!fractals || !offsets)) return fail(NBB_E_INVALID, "null argument");
    if ((flags & ~uint32_t(NBB_BATCH_NO_RESIDENT | NBB_BATCH_RESIDENT)) ||
        flags == (NBB_BATCH_NO_RESIDENT | NBB_BATCH_RESIDENT))
        return fail(NBB_E_INVALID, "unknown or conflicting batch flags");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const uint64_t kArenaLimit = uint64_t(1) << 36;
    for (uint32_t i = 0; i < count; ++i) {
        const nbb_fractal *F = fractals[i];
        if (!F) return fail(NBB_E_INVALID, "null descriptor in the batch");
        if (F->device != dev) return fail(NBB_E_INVALID, "descriptor belongs to another device");
        if (offsets[i] % 16) return fail(NBB_E_INVALID, "instance offsets must be multiples of 16");
        if (offsets[i] >= kArenaLimit || F->f.cells > kArenaLimit)
            return fail(NBB_E_RANGE, "instance offset beyond 2^36");
    }
    // Ranges must not overlap: check them in offset order.
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return offsets[x] < offsets[y]; });
    nbb_batch *B = new (std::nothrow) nbb_batch;
    if (!B) return fail(NBB_E_NOMEM, "host allocation failed");
    B->device = dev;
    B->count = count;
    for (uint32_t j = 0; j < count; ++j) {
        const uint32_t i = order[j];
        const uint64_t end = offsets[i] + fractals[i]->f.cells;
        if (j + 1 < count && end > offsets[order[j + 1]]) {
            delete B;
            return fail(NBB_E_INVALID, "instance ranges overlap");
        }
        B->cells += fractals[i]->f.cells;
        B->arena_bytes = std::max(B->arena_bytes, (end + 15) & ~uint64_t(15));
    }
    // Group the tiled instances by (k, s, offsets, tile plan).
    auto same_plan = [](const nbb_fractal *x, const nbb_fractal *y) {
        if (x->f.k != y->f.k || x->f.s != y->f.s) return false;
        for (uint32_t j = 0; j < x->f.k; ++j)
            if (x->f.ox[j] != y->f.ox[j] || x->f.oy[j] != y->f.oy[j]) return false;
        const TileParams &a = x->tp, &b = y->tp;
        return x->strategy == y->strategy && x->use_edges == y->use_edges && a.team == b.team && a.m == b.m &&
               a.W == b.W && a.lds_total == b.lds_total && a.halo_count == b.halo_count;
    };
    // Resident instances group by their resident plans.
    auto same_resident = [](const nbb_fractal *x, const nbb_fractal *y) {
        if (x->f.k != y->f.k || x->f.s != y->f.s) return false;
        for (uint32_t j = 0; j < x->f.k; ++j)
            if (x->f.ox[j] != y->f.ox[j] || x->f.oy[j] != y->f.oy[j]) return false;
        const TileParams &a = x->res_tp, &b = y->res_tp;
        return a.m == b.m && a.W == b.W && a.lds_total == b.lds_total && a.halo_count == b.halo_count;
    };
    // Instances keep the caller's order inside each group (nbb_batch_step_each
    // relies on it).
    struct Part {
        std::vector<const nbb_fractal *> reps;
        std::vector<std::vector<BatchInstance>> members;
        std::vector<std::vector<uint32_t>> index;
        void add(const nbb_fractal *F, uint32_t i, const BatchInstance &I,
                 const std::function<bool(const nbb_fractal *, const nbb_fractal *)> &same) {
            size_t g = 0;
            while (g < reps.size() && !same(reps[g], F)) ++g;
            if (g == reps.size()) {
                reps.push_back(F);
                members.emplace_back();
                index.emplace_back();
            }
            index[g].push_back(i);
            members[g].push_back(I);
        }
    } launch, res;
    // Small instances go to LDS when asked to, or by default when they hold
    // at least 1/8 of the tiled cells: beside a few large instances they are
    // cheap in the group launches, while a long resident launch takes issue
    // slots from every generation of those.
    bool use_resident = false;
    if (!(flags & NBB_BATCH_NO_RESIDENT)) {
        uint64_t tiled = 0, small = 0;
        for (uint32_t i = 0; i < count; ++i) {
            const nbb_fractal *F = fractals[i];
            if (F->strategy == NBB_STRATEGY_DIRECT) continue;
            uint32_t teams = 0;
            tiled += F->f.cells;
            if (resident_plan(F, &teams)) small += F->f.cells;
        }
        use_resident = (flags & NBB_BATCH_RESIDENT) ? small > 0 : (small && 8 * small >= tiled);
    }
    for (uint32_t i = 0; i < count; ++i) {
        const nbb_fractal *F = fractals[i];
        if (F->strategy == NBB_STRATEGY_DIRECT) {
            B->direct.push_back({F, offsets[i], i});
            continue;
        }
        uint32_t teams = 0;
        const TileParams *rp = use_resident ? resident_plan(F, &teams) : nullptr;
        const TileParams &tp = rp ? *rp : F->tp;
        BatchInstance I{};
        I.nbr = tp.nbr;
        I.base16 = uint32_t(offsets[i] >> 4);
        I.ntiles = tp.ntiles;
        I.tail_partial = (F->f.cells & 15) ? 1u : 0u;
        if (rp)
            res.add(F, i, I, same_resident);
        else
            launch.add(F, i, I, same_plan);
    }
    // One device allocation: per group the instance table, the records
    // (2 words per tile) and the neighbour table (8 words per tile); per
    // resident group its instance table.
    const size_t ng = launch.reps.size(), nr = res.reps.size();
    std::vector<size_t> off_inst(ng), off_rec(ng), off_nbr(ng), ntiles(ng);
    size_t total = 0;
    for (size_t g = 0; g < ng; ++g) {
        uint64_t t = 0;
        for (BatchInstance &I : launch.members[g]) {
            I.tile0 = uint32_t(t);
            t += I.ntiles;
        }
        if (t * 8 > (uint64_t(1) << 31)) {
            delete B;
            return fail(NBB_E_RANGE, "too many tiles in one group of the batch");
        }
        ntiles[g] = t;
        B->tiles += t;
        off_inst[g] = total;
        total += align256(launch.members[g].size() * sizeof(BatchInstance));
        off_rec[g] = total;
        total += align256(std::max<size_t>(t * 8, 1));
        off_nbr[g] = total;
        total += align256(std::max<size_t>(t * 32, 1));
    }
    size_t nres = 0;
    for (size_t g = 0; g < nr; ++g) {
        for (const BatchInstance &I : res.members[g]) B->tiles += I.ntiles;
        nres += res.members[g].size();
    }
    const size_t off_plans = total;
    total += nr ? align256(nr * sizeof(TileParams)) : 0;
    const size_t off_rinst = total;
    total += nres ? align256(nres * sizeof(ResidentInstance)) : 0;
    const size_t off_rsteps = total;
    total += nres ? align256(nres * sizeof(uint32_t)) : 0;
    if (fixed && total > fixed_cap) {
        delete B;
        return fail(NBB_E_RANGE, "batch tables (" + std::to_string(total) + " bytes) exceed the " +
                                     std::to_string(fixed_cap) + "-byte no-allocation scratch");
    }
    if (total && !fixed) {
        e = hipMalloc(&B->dtab.ptr, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete B;
            return e == hipErrorOutOfMemory ? fail(NBB_E_NOMEM, "batch table allocation failed")
                                            : hip_fail(e, "hipMalloc");
        }
        B->dtab.bytes = total;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = fixed ? reinterpret_cast<char *>(fixed) : static_cast<char *>(B->dtab.ptr);
    for (size_t g = 0; g < ng; ++g) {
        auto *inst = reinterpret_cast<BatchInstance *>(base + off_inst[g]);
        auto *rec = reinterpret_cast<uint32_t *>(base + off_rec[g]);
        auto *nbr = reinterpret_cast<uint32_t *>(base + off_nbr[g]);
        static_assert(sizeof(BatchInstance) % 4 == 0, "instance records upload as words");
        if (fixed) {
            e = launch_set_words(reinterpret_cast<uint32_t *>(inst),
                                 reinterpret_cast<const uint32_t *>(launch.members[g].data()),
                                 uint32_t(launch.members[g].size() * sizeof(BatchInstance) / 4), s);
        } else {
            e = hipMemcpyAsync(inst, launch.members[g].data(), launch.members[g].size() * sizeof(BatchInstance),
                               hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host table goes out of scope
        }
        if (e == hipSuccess)
            e = launch_batch_tiles(inst, uint32_t(launch.members[g].size()), uint32_t(ntiles[g]), rec, nbr, s);
        if (e != hipSuccess) {
            batch_free(B);
            return hip_fail(e, "batch table build");
        }
        BatchGroup G;
        G.tp = launch.reps[g]->tp;
        G.tp.nbr = nbr;
        G.tp.ntiles = uint32_t(ntiles[g]);
        G.tp.cells = 0;  // per instance, from the records
        G.rec = rec;
        const nbb_fractal *rep = launch.reps[g];
        if (rep->use_edges) {
            G.edges = true;
            G.ep = rep->ep;
            G.ep.nbr = nbr;
            G.ep.ntiles = uint32_t(ntiles[g]);
            G.BS = rep->edge.BS;
            G.nsrc = rep->edge.nsrc;
        }
        G.index = launch.index[g];
        uint64_t acc = 0;
        for (const BatchInstance &I : launch.members[g]) G.tiles_end.push_back(acc += I.ntiles);
        B->groups.push_back(std::move(G));
        B->cu_count = launch.reps[g]->cu_count;
    }
    if (nr) {
        // tiles per pass per plan: as many (up to 4) as the registers and LDS
        // allow for the plan's largest instance
        const uint32_t lds_budget = device_lds_per_group();
        std::vector<TileParams> plans(nr);
        std::vector<ResidentInstance> rinst;
        ResidentSet &R = B->resident;
        for (size_t g = 0; g < nr; ++g) {
            plans[g] = res.reps[g]->res_tp;
            uint32_t most = 1;
            for (const BatchInstance &I : res.members[g]) most = std::max(most, I.ntiles);
            uint32_t teams = 1;
            for (uint32_t t : {4u, 2u})
                if (t <= most && resident_fits(plans[g], t) && resident_lds_bytes(plans[g], most, t) <= lds_budget) {
                    teams = t;
                    break;
                }
            R.lds = std::max(R.lds, resident_lds_bytes(plans[g], most, teams));
            for (size_t j = 0; j < res.members[g].size(); ++j) {
                const BatchInstance &I = res.members[g][j];
                rinst.push_back({I.nbr, I.base16, I.ntiles, uint32_t(g), teams});
                R.index.push_back(res.index[g][j]);
                R.passes.push_back((I.ntiles + teams - 1) / teams);
            }
        }
        auto *dplans = reinterpret_cast<TileParams *>(base + off_plans);
        auto *dinst = reinterpret_cast<ResidentInstance *>(base + off_rinst);
        e = hipMemcpyAsync(dplans, plans.data(), nr * sizeof(TileParams), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dinst, rinst.data(), rinst.size() * sizeof(ResidentInstance), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host tables go out of scope
        if (e != hipSuccess) {
            batch_free(B);
            return hip_fail(e, "batch table build");
        }
        R.plans = dplans;
        R.inst = dinst;
        R.steps = reinterpret_cast<uint32_t *>(base + off_rsteps);
    }
    for (const BatchDirect &d : B->direct) B->cu_count = d.f->cu_count;
    // a side stream if the resident launch has group or direct launches beside it
    if (!B->resident.index.empty() && (!B->groups.empty() || !B->direct.empty())) {
        e = resident_stream(dev, &B->side);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            B->side = nullptr;
            batch_free(B);
            return hip_fail(e, "batch stream");
        }
    }
    if (!fixed && B->groups.size() > 1) {
        const size_t ns = std::min<size_t>(B->groups.size() - 1, kGroupStreams);
        e = hipEventCreateWithFlags(&B->gfork, hipEventDisableTiming);
        for (size_t i = 0; i < ns && e == hipSuccess; ++i) {
            hipStream_t gs = nullptr;
            hipEvent_t ev = nullptr;
            e = device_stream(dev, int(1 + i), &gs);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) {
                B->gstream.push_back(gs);
                B->gjoin.push_back(ev);
            }
        }
        if (e != hipSuccess) {
            batch_free(B);
            return hip_fail(e, "batch group streams");
        }
    }
    *out = B;
    return NBB_OK;
}

nbb_status nbb_batch_create_ex(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                               uint32_t flags, void *stream, nbb_batch **out) {
    return batch_create(fractals, offsets, count, flags, stream, nullptr, 0, out);
}

void nbb_batch_destroy(nbb_batch *B) {
    if (B) batch_free(B);
}

nbb_status nbb_batch_query(const nbb_batch *B, nbb_batch_info *info) {
    if (!B || !info) return fail(NBB_E_INVALID, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->instances = B->count;
    info->groups = uint32_t(B->groups.size());
    info->direct = uint32_t(B->direct.size());
    info->resident = uint32_t(B->resident.index.size());
    info->cells = B->cells;
    info->tiles = B->tiles;
    info->arena_bytes = B->arena_bytes;
    info->device_table_bytes = B->dtab.bytes;
    return NBB_OK;
}

// Enqueues the resident launch (instance i of the batch takes steps[i]
// generations, or steps_all if steps is NULL; the per-instance counts go to
// the batch's device array first): on the caller's stream if nothing else
// runs, else on the side stream, forked from it here; batch_join_resident
// joins it back.  *launched tells whether anything was enqueued.
static hipError_t batch_fork_resident(const nbb_batch *B, uint8_t *a, uint8_t *b, uint32_t rule,
                                      const uint32_t *steps, uint32_t steps_all, hipStream_t s, bool *launched_) {
    *launched_ = false;
    const ResidentSet &R = B->resident;
    const uint32_t count = uint32_t(R.index.size());
    if (!count) return hipSuccess;
    std::vector<uint32_t> n;
    bool any = steps_all != 0;
    if (steps) {
        n.resize(count);
        for (uint32_t j = 0; j < count; ++j) any |= (n[j] = steps[R.index[j]]) != 0;
    }
    if (!any) return hipSuccess;
    hipStream_t rs = s;
    if (B->side) {
        hipError_t e = hipEventRecord(B->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(B->side, B->fork, 0);
        if (e != hipSuccess) return e;
        rs = B->side;
    }
    if (steps) {
        hipError_t e = launch_set_words(R.steps, n.data(), count, rs);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_step_resident(R.plans, R.inst, count, steps ? R.steps : nullptr, steps_all, R.lds, a, b,
                                        rule, rs);
    if (e == hipSuccess && B->side) e = hipEventRecord(B->join, B->side);
    *launched_ = e == hipSuccess;
    return e;
}
static hipError_t batch_join_resident(const nbb_batch *B, hipStream_t s, bool launched_) {
    return (launched_ && B->side) ? hipStreamWaitEvent(s, B->join, 0) : hipSuccess;
}
// The group streams start after the work enqueued on s so far; group k's
// launches go to batch_group_stream(B, k, s); batch_join_groups makes s wait
// for all of them.  Groups touch disjoint instance ranges of the arenas
// (a window read past a block's bytes may reach into another instance's
// range, but those bytes are not used), so they need no order between them.
static hipError_t batch_fork_groups(const nbb_batch *B, hipStream_t s) {
    if (B->gstream.empty()) return hipSuccess;
    hipError_t e = hipEventRecord(B->gfork, s);
    for (size_t i = 0; i < B->gstream.size() && e == hipSuccess; ++i) e = hipStreamWaitEvent(B->gstream[i], B->gfork, 0);
    return e;
}
static hipStream_t batch_group_stream(const nbb_batch *B, size_t k, hipStream_t s) {
    return (k == 0 || B->gstream.empty()) ? s : B->gstream[(k - 1) % B->gstream.size()];
}
static hipError_t batch_join_groups(const nbb_batch *B, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < B->gstream.size() && e == hipSuccess; ++i) {
        e = hipEventRecord(B->gjoin[i], B->gstream[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, B->gjoin[i], 0);
    }
    return e;
}

nbb_status nbb_batch_step(const nbb_batch *B, uint8_t *a, uint8_t *b, uint64_t arena_len, uint32_t steps,
                          uint32_t rule, int *result_in_b, void *stream) {
    if (!B) return fail(NBB_E_INVALID, "null batch");
    if (B->count && (!a || !b)) return fail(NBB_E_INVALID, "null arena");
    if (arena_len < B->arena_bytes) return fail(NBB_E_INVALID, "arena shorter than the batch needs");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "arenas must be 16-byte aligned");
    if (B->count && overlap(a, b, arena_len)) return fail(NBB_E_INVALID, "arenas overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != B->device) return fail(NBB_E_INVALID, "batch belongs to another device");
    if (result_in_b) *result_in_b = int(steps & 1);
    if (!steps) return NBB_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool res_launched = false;
    e = batch_fork_resident(B, a, b, rule, nullptr, steps, s, &res_launched);
    if (e != hipSuccess) return hip_fail(e, "batch resident step launch");
    e = batch_fork_groups(B, s);
    if (e != hipSuccess) return hip_fail(e, "batch group fork");
    // each group takes all its generations on its stream
    for (size_t k = 0; k < B->groups.size() && e == hipSuccess; ++k) {
        const BatchGroup &G = B->groups[k];
        const hipStream_t gs = batch_group_stream(B, k, s);
        uint8_t *in = a, *out = b;
        for (uint32_t i = 0; i < steps && e == hipSuccess; ++i) {
            e = G.edges ? launch_step_edges(G.ep, G.BS, G.nsrc, in, out, arena_len, rule, G.rec, B->cu_count, gs)
                        : launch_step_tiled_batch(G.tp, G.rec, in, out, rule, B->cu_count, gs);
            std::swap(in, out);
        }
    }
    const char *what = "batch step launch";
    for (size_t j = 0; j < B->direct.size() && e == hipSuccess; ++j) {
        const nbb_fractal *F = B->direct[j].f;
        const uint64_t off = B->direct[j].offset;
        uint8_t *in = a, *out = b;
        for (uint32_t i = 0; i < steps && e == hipSuccess; ++i) {
            e = launch_step_direct(F->mp, F->lam_words, F->nu_halves, in + off, out + off, rule,
                                   map_grid(F, F->f.cells), s);
            std::swap(in, out);
        }
        what = "batch direct step launch";
    }
    // joined also after a failed launch, so that s does not run ahead of
    // what was enqueued on the other streams
    const hipError_t ej = batch_join_groups(B, s);
    if (e != hipSuccess) return hip_fail(e, what);
    if (ej != hipSuccess) return hip_fail(ej, "batch group join");
    e = batch_join_resident(B, s, res_launched);
    return e == hipSuccess ? NBB_OK : hip_fail(e, "batch resident join");
}

nbb_status nbb_batch_step_each(const nbb_batch *B, uint8_t *a, uint8_t *b, uint64_t arena_len,
                               const uint32_t *steps, uint32_t rule, void *stream) {
    if (!B) return fail(NBB_E_INVALID, "null batch");
    if (B->count && (!a || !b || !steps)) return fail(NBB_E_INVALID, "null argument");
    if (arena_len < B->arena_bytes) return fail(NBB_E_INVALID, "arena shorter than the batch needs");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "arenas must be 16-byte aligned");
    if (B->count && overlap(a, b, arena_len)) return fail(NBB_E_INVALID, "arenas overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != B->device) return fail(NBB_E_INVALID, "batch belongs to another device");
    uint32_t most = 0;
    for (const BatchGroup &G : B->groups)
        for (size_t j = 0; j < G.index.size(); ++j) {
            if (j && steps[G.index[j]] > steps[G.index[j - 1]])
                return fail(NBB_E_INVALID, "step counts must not increase within a group of the batch");
            most = std::max(most, steps[G.index[j]]);
        }
    for (const BatchDirect &d : B->direct) most = std::max(most, steps[d.index]);
    // Generation g steps, in each group, the prefix of instances with more
    // than g steps; instance i's state alternates a -> b -> a ... like the
    // whole batch's, so its result ends in b iff steps[i] is odd.
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool res_launched = false;
    e = batch_fork_resident(B, a, b, rule, steps, 0, s, &res_launched);
    if (e != hipSuccess) return hip_fail(e, "batch resident step launch");
    e = batch_fork_groups(B, s);
    if (e != hipSuccess) return hip_fail(e, "batch group fork");
    for (size_t k = 0; k < B->groups.size() && e == hipSuccess; ++k) {
        const BatchGroup &G = B->groups[k];
        const hipStream_t gs = batch_group_stream(B, k, s);
        size_t live = G.index.size();
        uint8_t *in = a, *out = b;
        for (uint32_t g = 0; g < most && e == hipSuccess; ++g) {
            while (live && steps[G.index[live - 1]] <= g) --live;
            if (!live) break;
            const uint32_t nt = uint32_t(G.tiles_end[live - 1]);
            if (G.edges) {
                EdgeParams E = G.ep;
                E.ntiles = nt;
                e = launch_step_edges(E, G.BS, G.nsrc, in, out, arena_len, rule, G.rec, B->cu_count, gs);
            } else {
                TileParams T = G.tp;
                T.ntiles = nt;
                e = launch_step_tiled_batch(T, G.rec, in, out, rule, B->cu_count, gs);
            }
            std::swap(in, out);
        }
    }
    const char *what = "batch step launch";
    for (size_t j = 0; j < B->direct.size() && e == hipSuccess; ++j) {
        const BatchDirect &d = B->direct[j];
        const nbb_fractal *F = d.f;
        uint8_t *in = a, *out = b;
        for (uint32_t g = 0; g < steps[d.index] && e == hipSuccess; ++g) {
            e = launch_step_direct(F->mp, F->lam_words, F->nu_halves, in + d.offset, out + d.offset, rule,
                                   map_grid(F, F->f.cells), s);
            std::swap(in, out);
        }
        what = "batch direct step launch";
    }
    const hipError_t ej = batch_join_groups(B, s);
    if (e != hipSuccess) return hip_fail(e, what);
    if (ej != hipSuccess) return hip_fail(ej, "batch group join");
    e = batch_join_resident(B, s, res_launched);
    if (e != hipSuccess) return hip_fail(e, "batch resident join");
    return NBB_OK;
}

// ---- tile plans of a batch chosen by measurement ----------------------------
// Results kept for the process: (device, k, s, offsets, smallest and largest
// r of the set, rule form) -> (strategy, tile level).
static std::mutex g_tune_mu;
static std::map<std::vector<uint32_t>, std::pair<uint32_t, uint32_t>> g_tune_cache;

nbb_status nbb_batch_autotune(nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count, uint8_t *a,
                              uint8_t *b, uint64_t arena_len, uint32_t steps, uint32_t rule, uint32_t flags,
                              void *stream) {
    if (count && (!fractals || !offsets || !a || !b)) return fail(NBB_E_INVALID, "null argument");
    if (steps == 0) return fail(NBB_E_INVALID, "steps must be >= 1");
    if (flags & ~uint32_t(NBB_TUNE_NO_CACHE)) return fail(NBB_E_INVALID, "unknown flag bits");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "arenas must be 16-byte aligned");
    if (count && overlap(a, b, arena_len)) return fail(NBB_E_INVALID, "arenas overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    for (uint32_t i = 0; i < count; ++i)
        if (!fractals[i]) return fail(NBB_E_INVALID, "null descriptor in the batch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    // the sets: instances of one fractal (k, s, offsets) that the tiled step supports
    auto same_fractal = [](const Fractal &x, const Fractal &y) {
        if (x.k != y.k || x.s != y.s) return false;
        for (uint32_t j = 0; j < x.k; ++j)
            if (x.ox[j] != y.ox[j] || x.oy[j] != y.oy[j]) return false;
        return true;
    };
    std::vector<std::vector<uint32_t>> sets;
    for (uint32_t i = 0; i < count; ++i) {
        if (!tiled_supported(fractals[i]->f)) continue;
        size_t g = 0;
        while (g < sets.size() && !same_fractal(fractals[sets[g][0]]->f, fractals[i]->f)) ++g;
        if (g == sets.size()) sets.emplace_back();
        sets[g].push_back(i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    nbb_status st = NBB_OK;
    for (const std::vector<uint32_t> &set : sets) {
        std::vector<nbb_fractal *> desc;  // distinct descriptors of the set
        uint32_t rmin = 0xFFFFFFFFu, rmax = 0;
        for (uint32_t i : set) {
            nbb_fractal *F = fractals[i];
            if (std::find(desc.begin(), desc.end(), F) == desc.end()) desc.push_back(F);
            rmin = std::min(rmin, F->f.r);
            rmax = std::max(rmax, F->f.r);
        }
        const Fractal &f0 = desc[0]->f;
        std::vector<uint32_t> key = {uint32_t(dev), f0.k, f0.s, rmin, rmax, uint32_t(edges_rule_kind(rule))};
        for (uint32_t j = 0; j < f0.k; ++j) {
            key.push_back(uint32_t(f0.ox[j]));
            key.push_back(uint32_t(f0.oy[j]));
        }
        auto configure_all = [&](uint32_t strategy, uint32_t m) {
            for (nbb_fractal *F : desc) {
                nbb_status c = nbb_configure(F, strategy, m);
                if (c != NBB_OK) return c;
            }
            return NBB_OK;
        };
        std::pair<uint32_t, uint32_t> best{0, 0};
        bool cached = false;
        if (!(flags & NBB_TUNE_NO_CACHE)) {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                best = it->second;
                cached = true;
            }
        }
        if (!cached) {
            // candidates: every tile level up to the set's smallest r whose
            // tiles hold at least 64 cells (or the largest level), in the
            // edge-record and the byte-scatter form
            std::vector<uint64_t> offs;
            std::vector<const nbb_fractal *> inst;
            for (uint32_t i : set) {
                offs.push_back(offsets[i]);
                inst.push_back(fractals[i]);
            }
            float best_ms = -1.0f;
            uint64_t K = 1;
            for (uint32_t m = 1; m <= rmin && st == NBB_OK; ++m) {
                K *= f0.k;
                if (K < 64 && m < rmin) continue;
                for (uint32_t strategy : {NBB_STRATEGY_TILED_EDGE, NBB_STRATEGY_TILED_BOX}) {
                    if (configure_all(strategy, m) != NBB_OK) continue;  // does not fit: skip it
                    nbb_batch *B = nullptr;
                    st = batch_create(inst.data(), offs.data(), uint32_t(inst.size()), NBB_BATCH_NO_RESIDENT,
                                      stream, nullptr, 0, &B);
                    if (st != NBB_OK) break;
                    float ms = 0.0f;
                    st = nbb_batch_step(B, a, b, arena_len, 1, rule, nullptr, stream);
                    if (st == NBB_OK && (e = hipEventRecord(e0, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
                    if (st == NBB_OK) st = nbb_batch_step(B, a, b, arena_len, steps, rule, nullptr, stream);
                    if (st == NBB_OK && (e = hipEventRecord(e1, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
                    if (st == NBB_OK && (e = hipEventSynchronize(e1)) != hipSuccess)
                        st = hip_fail(e, "hipEventSynchronize");
                    if (st == NBB_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
                        st = hip_fail(e, "hipEventElapsedTime");
                    batch_free(B);
                    if (st != NBB_OK) break;
                    if (best_ms < 0.0f || ms < best_ms) {
                        best_ms = ms;
                        best = {strategy, m};
                    }
                }
            }
            if (st != NBB_OK) break;
            if (best_ms < 0.0f) continue;  // nothing fits: the descriptors keep what they had
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune_cache[key] = best;
        }
        st = configure_all(best.first, best.second);
        if (st != NBB_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// ---- the batched step without allocation ---------------------------------
// The batch tables of nbb_batch_step_each_noalloc live in this array, one
// copy per device (it is a device variable), held until the process ends.
// Host code never passes the array's name to a kernel or a copy: on the host
// it is only a stand-in for the symbol; the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) uint8_t scratch[NBB_NOALLOC_SCRATCH_BYTES];

static nbb_status scratch_address(int dev, uint8_t **out) {
    static std::mutex mu;
    static std::vector<uint8_t *> addr;  // per device, null until looked up
    std::lock_guard<std::mutex> lock(mu);
    if (addr.size() <= size_t(dev)) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        addr[dev] = static_cast<uint8_t *>(p);
    }
    *out = addr[dev];
    return NBB_OK;
}

nbb_status nbb_batch_step_each_noalloc(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                                       uint8_t *a, uint8_t *b, uint64_t arena_len, const uint32_t *steps,
                                       uint32_t rule, void *stream) {
    // the arena checks of nbb_batch_step_each, before any table is enqueued
    if (count && (!fractals || !offsets || !steps || !a || !b)) return fail(NBB_E_INVALID, "null argument");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "arenas must be 16-byte aligned");
    if (count && overlap(a, b, arena_len)) return fail(NBB_E_INVALID, "arenas overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    for (uint32_t i = 0; i < count; ++i) {
        if (!fractals[i]) return fail(NBB_E_INVALID, "null descriptor in the batch");
        const uint64_t end = offsets[i] + fractals[i]->f.cells;  // offsets < 2^36 are checked below
        if (offsets[i] >= (uint64_t(1) << 36) || ((end + 15) & ~uint64_t(15)) > arena_len)
            return offsets[i] >= (uint64_t(1) << 36) ? fail(NBB_E_RANGE, "instance offset beyond 2^36")
                                                     : fail(NBB_E_INVALID, "arena shorter than the batch needs");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    uint8_t *tables = nullptr;
    nbb_status st = scratch_address(dev, &tables);
    if (st != NBB_OK) return st;
    nbb_batch *B = nullptr;
    st = batch_create(fractals, offsets, count, NBB_BATCH_NO_RESIDENT, stream, tables, NBB_NOALLOC_SCRATCH_BYTES,
                      &B);
    if (st != NBB_OK) return st;
    st = nbb_batch_step_each(B, a, b, arena_len, steps, rule, stream);
    batch_free(B);  // host bookkeeping only: B owns no device memory
    return st;
}

uint64_t nbb_bbox_pitch(const nbb_fractal *F) { return F ? box_pitch(F->f) : 0; }

nbb_status nbb_lambda_method(const nbb_fractal *F, uint32_t method, const uint32_t *idx, uint64_t count,
                             int32_t *x, int32_t *y, void *stream) {
    if (!F) return fail(NBB_E_INVALID, "null descriptor");
    if (method > NBB_MAP_MFMA) return fail(NBB_E_INVALID, "unknown map method");
    if (method == NBB_MAP_MFMA && !F->ml.ktiles)
        return fail(NBB_E_INVALID, "the matrix-core lambda needs r*k <= 192 and n <= 2^28");
    if (count == 0) return NBB_OK;
    if (!x || !y) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (method) {
        case NBB_MAP_LUT:
            return launched(launch_lambda(F->mp, F->lam_words, idx, count, x, y, map_grid(F, count), s),
                            "lambda launch");
        case NBB_MAP_DIGITS:
            return launched(launch_lambda_digits(F->mp, idx, count, x, y, map_grid(F, count), s), "lambda launch");
        default: {
            const uint64_t groups = (count + 255) / 256;
            const int grid = int(std::max<uint64_t>(1, std::min<uint64_t>(groups, uint64_t(F->cu_count) * 8)));
            return launched(launch_lambda_mfma(F->mp, F->ml, idx, count, x, y, grid, s), "lambda launch");
        }
    }
}

nbb_status nbb_lambda(const nbb_fractal *F, const uint32_t *idx, uint64_t count, int32_t *x, int32_t *y,
                      void *stream) {
    return nbb_lambda_method(F, NBB_MAP_LUT, idx, count, x, y, stream);
}

nbb_status nbb_nu_method(const nbb_fractal *F, uint32_t method, const int32_t *x, const int32_t *y, uint64_t count,
                         uint32_t *idx, void *stream) {
    if (!F) return fail(NBB_E_INVALID, "null descriptor");
    if (method > NBB_MAP_MFMA) return fail(NBB_E_INVALID, "unknown map method");
    if (method == NBB_MAP_MFMA && !F->ml.ktiles)
        return fail(NBB_E_INVALID, "the matrix-core nu needs r*k <= 192 and n <= 2^28");
    if (count == 0) return NBB_OK;
    if (!x || !y || !idx) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (method == NBB_MAP_DIGITS)
        return launched(launch_nu_digits(F->mp, x, y, count, idx, map_grid(F, count), s), "nu launch");
    if (method == NBB_MAP_MFMA)
        return launched(launch_nu_mfma(F->mp, F->ml, x, y, count, idx, map_grid(F, count), s), "nu launch");
    return launched(launch_nu(F->mp, F->nu_halves, x, y, count, idx, map_grid(F, count), s), "nu launch");
}

nbb_status nbb_nu(const nbb_fractal *F, const int32_t *x, const int32_t *y, uint64_t count, uint32_t *idx,
                  void *stream) {
    return nbb_nu_method(F, NBB_MAP_LUT, x, y, count, idx, stream);
}

static uint32_t threshold24(double p) {
    if (p >= 1.0) return 1u << 24;
    return uint32_t(p * 16777216.0);
}

nbb_status nbb_init_compact(const nbb_fractal *F, uint8_t *state, uint64_t len, uint64_t seed, double p,
                            void *stream) {
    if (!F || !state) return fail(NBB_E_INVALID, "null argument");
    if (len != F->f.cells) return fail(NBB_E_INVALID, "len must equal k^r");
    if (!aligned16(state)) return fail(NBB_E_INVALID, "state must be 16-byte aligned");
    if (!(p >= 0.0 && p <= 1.0)) return fail(NBB_E_INVALID, "p must lie in [0, 1]");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    return launched(launch_init_compact(F->mp, F->lam_words, state, seed, threshold24(p),
                                        map_grid(F, (len + 15) / 16), static_cast<hipStream_t>(stream)),
                    "init launch");
}

nbb_status nbb_init_bbox(const nbb_fractal *F, uint8_t *state, uint64_t pitch, uint64_t len, uint64_t seed,
                         double p, void *stream) {
    if (!F) return fail(NBB_E_INVALID, "null descriptor");
    nbb_status st = check_box_args(F, state, pitch, len);
    if (st != NBB_OK) return st;
    if (!(p >= 0.0 && p <= 1.0)) return fail(NBB_E_INVALID, "p must lie in [0, 1]");
    st = check_device(F);
    if (st != NBB_OK) return st;
    BoxParams B = F->bp;
    B.pitch = pitch;
    return launched(launch_init_box(B, state, seed, threshold24(p), static_cast<hipStream_t>(stream)),
                    "box init launch");
}

nbb_status nbb_step_compact(const nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                            uint32_t rule, int *result_in_b, void *stream) {
    if (!F || !a || !b) return fail(NBB_E_INVALID, "null argument");
    if (len != F->f.cells) return fail(NBB_E_INVALID, "len must equal k^r");
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (!aligned16(a) || !aligned16(b)) return fail(NBB_E_INVALID, "state buffers must be 16-byte aligned");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    nbb_status st = check_device(F);
    if (st != NBB_OK) return st;
    if (result_in_b) *result_in_b = int(steps & 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *in = a, *out = b;
    if (F->strategy == NBB_STRATEGY_TEMPORAL) {
        // L launches of up to h generations each; the result must end in b
        // iff steps is odd, so L takes the parity of steps (one more launch
        // when needed: then L < steps, so every launch still has one)
        const uint32_t h = F->tmp.h;
        uint32_t L = (steps + h - 1) / h;
        if ((L & 1) != (steps & 1)) ++L;
        for (uint32_t i = 0; i < L; ++i) {
            const uint32_t g = steps / L + (i < steps % L ? 1u : 0u);
            hipError_t e = launch_step_temporal(F->tmp, in, out, rule, g, s);
            if (e != hipSuccess) return hip_fail(e, "temporal step launch");
            std::swap(in, out);
        }
    } else if (F->use_edges) {
        for (uint32_t i = 0; i < steps; ++i) {
            hipError_t e = launch_step_edges(F->ep, F->edge.BS, F->edge.nsrc, in, out, F->f.cells, rule, nullptr, F->cu_count,
                                             s);
            if (e != hipSuccess) return hip_fail(e, "edge step launch");
            std::swap(in, out);
        }
    } else if (F->strategy != NBB_STRATEGY_DIRECT) {
        for (uint32_t i = 0; i < steps; ++i) {
            hipError_t e = launch_step_tiled(F->mp, F->tp, in, out, rule, F->cu_count, s);
            if (e != hipSuccess) return hip_fail(e, "tiled step launch");
            std::swap(in, out);
        }
    } else {
        const int grid = map_grid(F, len);
        for (uint32_t i = 0; i < steps; ++i) {
            hipError_t e = launch_step_direct(F->mp, F->lam_words, F->nu_halves, in, out, rule, grid, s);
            if (e != hipSuccess) return hip_fail(e, "direct step launch");
            std::swap(in, out);
        }
    }
    return NBB_OK;
}

nbb_status nbb_step_bbox(const nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t pitch, uint64_t len,
                         uint32_t steps, uint32_t rule, int *result_in_b, void *stream) {
    if (!F || !b) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_box_args(F, a, pitch, len);
    if (st != NBB_OK) return st;
    if (!aligned16(b)) return fail(NBB_E_INVALID, "box state must be 16-byte aligned");
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    st = check_device(F);
    if (st != NBB_OK) return st;
    if (result_in_b) *result_in_b = int(steps & 1);
    BoxParams B = F->bp;
    B.pitch = pitch;
    uint8_t *in = a, *out = b;
    for (uint32_t i = 0; i < steps; ++i) {
        hipError_t e = launch_step_box(B, in, out, rule, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "box step launch");
        std::swap(in, out);
    }
    return NBB_OK;
}

nbb_status nbb_step_lambda(const nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t pitch, uint64_t len,
                           uint32_t steps, uint32_t rule, int *result_in_b, void *stream) {
    if (!F || !b) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_box_args(F, a, pitch, len);
    if (st != NBB_OK) return st;
    if (!aligned16(b)) return fail(NBB_E_INVALID, "box state must be 16-byte aligned");
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    st = check_device(F);
    if (st != NBB_OK) return st;
    if (result_in_b) *result_in_b = int(steps & 1);
    if (steps == 0) return NBB_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // only fractal cells are written: b's other cells must start at 0
    hipError_t e = launch_fill_zero(b, len, s);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    const int grid = map_grid(F, F->f.cells);
    uint8_t *in = a, *out = b;
    for (uint32_t i = 0; i < steps; ++i) {
        e = launch_step_lambda(F->mp, F->lam_words, in, out, pitch, rule, grid, s);
        if (e != hipSuccess) return hip_fail(e, "lambda step launch");
        std::swap(in, out);
    }
    return NBB_OK;
}

uint64_t nbb_blocked_bytes(const nbb_fractal *F) {
    if (!F || F->strategy == NBB_STRATEGY_DIRECT) return 0;
    return F->tile.ntiles * uint64_t(F->tile.S) * F->tile.S;
}

static nbb_status check_blocked(const nbb_fractal *F, const void *blocked, uint64_t len) {
    if (F->strategy == NBB_STRATEGY_DIRECT) return fail(NBB_E_INVALID, "the blocked layout needs a tiled plan");
    if (!blocked) return fail(NBB_E_INVALID, "null argument");
    if (len != nbb_blocked_bytes(F)) return fail(NBB_E_INVALID, "len must equal nbb_blocked_bytes");
    if (!aligned16(blocked)) return fail(NBB_E_INVALID, "blocked state must be 16-byte aligned");
    return NBB_OK;
}

nbb_status nbb_blocked_from_compact(const nbb_fractal *F, const uint8_t *compact, uint8_t *blocked, uint64_t len,
                                    void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_blocked(F, blocked, len);
    if (st != NBB_OK) return st;
    st = check_device(F);
    if (st != NBB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_fill_zero(blocked, len & ~uint64_t(15), s);
    if (e == hipSuccess) e = launch_fill_tail(blocked + (len & ~uint64_t(15)), uint32_t(len & 15), s);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    return launched(launch_blocked_scatter(F->tp, compact, blocked, F->f.cells, map_grid(F, F->f.cells), s),
                    "blocked scatter launch");
}

nbb_status nbb_blocked_to_compact(const nbb_fractal *F, const uint8_t *blocked, uint64_t len, uint8_t *compact,
                                  void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_blocked(F, blocked, len);
    if (st != NBB_OK) return st;
    st = check_device(F);
    if (st != NBB_OK) return st;
    return launched(launch_blocked_gather(F->tp, blocked, compact, F->f.cells, map_grid(F, F->f.cells),
                                          static_cast<hipStream_t>(stream)),
                    "blocked gather launch");
}

nbb_status nbb_step_blocked(const nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                            uint32_t rule, int *result_in_b, void *stream) {
    if (!F || !a || !b) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_blocked(F, a, len);
    if (st == NBB_OK) st = check_blocked(F, b, len);
    if (st != NBB_OK) return st;
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    st = check_device(F);
    if (st != NBB_OK) return st;
    if (result_in_b) *result_in_b = int(steps & 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *in = a, *out = b;
    for (uint32_t i = 0; i < steps; ++i) {
        hipError_t e = launch_step_blocked(F->tp, in, out, rule, F->cu_count, s);
        if (e != hipSuccess) return hip_fail(e, "blocked step launch");
        std::swap(in, out);
    }
    return NBB_OK;
}

uint64_t nbb_packed_bytes(const nbb_fractal *F) { return F ? (F->f.cells + 31) / 32 * 4 : 0; }

static nbb_status check_packed(const nbb_fractal *F, const void *packed, uint64_t len) {
    if (F->strategy == NBB_STRATEGY_DIRECT) return fail(NBB_E_INVALID, "the packed state needs a tiled plan");
    if (!packed) return fail(NBB_E_INVALID, "null argument");
    if (len != nbb_packed_bytes(F)) return fail(NBB_E_INVALID, "len must equal nbb_packed_bytes");
    if (reinterpret_cast<uintptr_t>(packed) & 3) return fail(NBB_E_INVALID, "packed state must be 4-byte aligned");
    return NBB_OK;
}

nbb_status nbb_pack(const nbb_fractal *F, const uint8_t *compact, uint8_t *packed, uint64_t len, void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_packed(F, packed, len);
    if (st == NBB_OK) st = check_device(F);
    if (st != NBB_OK) return st;
    return launched(launch_pack_bits(compact, reinterpret_cast<uint32_t *>(packed), F->f.cells,
                                     map_grid(F, len / 4), static_cast<hipStream_t>(stream)),
                    "pack launch");
}

nbb_status nbb_unpack(const nbb_fractal *F, const uint8_t *packed, uint64_t len, uint8_t *compact, void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_packed(F, packed, len);
    if (st == NBB_OK) st = check_device(F);
    if (st != NBB_OK) return st;
    return launched(launch_unpack_bits(reinterpret_cast<const uint32_t *>(packed), compact, F->f.cells,
                                       map_grid(F, len / 4), static_cast<hipStream_t>(stream)),
                    "unpack launch");
}

// The 32-phase copy of the plan's lut0 for the packed step (built on first
// use, kept with the descriptor, rebuilt after a change of plan).
static nbb_status packed_table(const nbb_fractal *F, const uint16_t **lut, uint32_t *stride) {
    std::lock_guard<std::mutex> lock(F->pk_mu);
    const TilePlan &P = F->tile;
    if (!F->dpk.ptr || F->pk_m != P.m || F->pk_W != P.W || F->pk_team != P.team) {
        blob_free(&F->dpk);
        const uint32_t K = P.K, S = 32 * ((K + 62) / 32);
        std::vector<uint16_t> t(size_t(32) * S, uint16_t(P.dummy));
        for (uint32_t p = 0; p < 32; ++p)
            for (uint32_t j = p; j < p + K; ++j) t[size_t(p) * S + j] = P.lut0p[j - p];  // phase-0 copy
        const void *src[1] = {t.data()};
        const size_t bytes[1] = {t.size() * 2};
        void *dst[1];
        nbb_status st = upload(&F->dpk, src, bytes, 1, dst);
        if (st != NBB_OK) return st;
        F->pk_stride = S;
        F->pk_m = P.m;
        F->pk_W = P.W;
        F->pk_team = P.team;
    }
    *lut = static_cast<const uint16_t *>(F->dpk.ptr);
    *stride = F->pk_stride;
    return NBB_OK;
}

nbb_status nbb_step_packed(const nbb_fractal *F, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                           uint32_t rule, int *result_in_b, void *stream) {
    if (!F || !a || !b) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_packed(F, a, len);
    if (st == NBB_OK) st = check_packed(F, b, len);
    if (st != NBB_OK) return st;
    if (overlap(a, b, len)) return fail(NBB_E_INVALID, "a and b overlap");
    if (rule & ~kRuleMask) return fail(NBB_E_INVALID, "rule uses bits outside 0-8, 16-24 and 31");
    if (!packed_fits(F->tp)) return fail(NBB_E_INVALID, "the tile plan exceeds the packed step's limits");
    st = check_device(F);
    if (st != NBB_OK) return st;
    if (result_in_b) *result_in_b = int(steps & 1);
    if (!steps) return NBB_OK;
    const uint16_t *lut = nullptr;
    uint32_t stride = 0;
    st = packed_table(F, &lut, &stride);
    if (st != NBB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *in = reinterpret_cast<uint32_t *>(a), *out = reinterpret_cast<uint32_t *>(b);
    for (uint32_t i = 0; i < steps; ++i) {
        hipError_t e = launch_step_packed(F->tp, lut, stride, in, out, rule, F->cu_count, s);
        if (e != hipSuccess) return hip_fail(e, "packed step launch");
        std::swap(in, out);
    }
    return NBB_OK;
}

nbb_status nbb_expand(const nbb_fractal *F, const uint8_t *compact, uint8_t *bbox, uint64_t pitch, uint64_t len,
                      void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    nbb_status st = check_box_args(F, bbox, pitch, len);
    if (st != NBB_OK) return st;
    st = check_device(F);
    if (st != NBB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_fill_zero(bbox, len, s);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    return launched(launch_expand(F->mp, F->lam_words, compact, bbox, pitch, map_grid(F, F->f.cells), s),
                    "expand launch");
}

nbb_status nbb_gather(const nbb_fractal *F, const uint8_t *bbox, uint64_t pitch, uint8_t *compact, uint64_t len,
                      void *stream) {
    if (!F || !compact) return fail(NBB_E_INVALID, "null argument");
    if (len != F->f.cells) return fail(NBB_E_INVALID, "len must equal k^r");
    nbb_status st = check_box_args(F, bbox, pitch, F->f.n * pitch);
    if (st != NBB_OK) return st;
    st = check_device(F);
    if (st != NBB_OK) return st;
    return launched(launch_gather(F->mp, F->lam_words, bbox, pitch, compact, map_grid(F, len),
                                  static_cast<hipStream_t>(stream)),
                    "gather launch");
}

}  // extern "C"
