/*
 * CPU oracle for compact NBB-fractal cellular automata.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * library.
 *
 * Everything here is written as the plain definition, in the paper's terms,
 * with no blocking, tiling or other reordering:
 *
 *   - An NBB fractal F^{k,s} at scale level r (sections 1 and 3) has k replica
 *     offsets o_0..o_{k-1} in [0,s)^2.  A cell (x,y) of the n x n box, n = s^r,
 *     is a member iff at every level mu < r its base-s digit pair
 *     (x_mu, y_mu) is one of the offsets.  |F| = k^r (eq. 1).
 *   - The replica id H at level mu is the position of (x_mu, y_mu) in the
 *     offset list (section 3.1, the look-up-table form of H).
 *   - lambda maps a compact index i = sum_mu d_mu k^mu to
 *     (x, y) = sum_mu o_{d_mu} s^mu; nu is its inverse on members
 *     (section 3: nu acts as the inverse of lambda) and reports "outside" for
 *     every other coordinate.
 *   - The paper's own 2D compact coordinates follow eqs. (3)-(8) with the
 *     exponent of tau read as floor(mu/2).
 *   - The automaton is a synchronous outer-totalistic rule on the Moore
 *     neighbourhood (section 4: Game of Life on the fractal); cells outside
 *     the fractal are dead and stay dead.
 *   - The initial state draws one SplitMix64 output per embedded cell
 *     (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
 *     OOPSLA 2014): cell key = y*n + x, output = mix(seed + (key+1)*gamma);
 *     the cell is alive iff it is a member and the top 24 bits of the output
 *     are below floor(p * 2^24).
 *
 * Rule word: bit c (c = 0..8) set = a dead cell with c live neighbours is born;
 * bit 16+c set = a live cell with c live neighbours survives.
 *
 * Compiled with gcc -O2 -fopenmp; loops over independent cells are split over
 * threads, which does not change any result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OUTSIDE (-1LL)

/* A fractal as the oracle sees it: the offsets plus the replica-id table of
 * section 3.1 (digit pair -> id, or -1 when the pair is not a replica). */
typedef struct {
    int64_t k, s, r, n, cells;
    int64_t ox[256], oy[256];
    int16_t id[256]; /* id[a + s*b] for digit pair (a, b) */
} orc_fractal;

static int64_t ipow(int64_t b, int64_t e) {
    int64_t p = 1;
    while (e-- > 0) p *= b;
    return p;
}

/* Fill *f; returns 0 on success, -1 on an argument the oracle does not accept. */
int orc_make(orc_fractal *f, int64_t k, int64_t s, const int32_t *offsets, int64_t r) {
    if (!f || !offsets || k < 1 || s < 2 || s > 16 || k > s * s || r < 0) return -1;
    memset(f, 0, sizeof(*f));
    f->k = k;
    f->s = s;
    f->r = r;
    f->n = ipow(s, r);
    f->cells = ipow(k, r);
    for (int64_t i = 0; i < 256; ++i) f->id[i] = -1;
    for (int64_t j = 0; j < k; ++j) {
        int64_t a = offsets[2 * j], b = offsets[2 * j + 1];
        if (a < 0 || a >= s || b < 0 || b >= s) return -1;
        if (f->id[a + s * b] != -1) return -1; /* replicas may not overlap */
        f->id[a + s * b] = (int16_t)j;
        f->ox[j] = a;
        f->oy[j] = b;
    }
    return 0;
}

size_t orc_fractal_size(void) { return sizeof(orc_fractal); }

/* Membership by the digit test. */
int orc_member(const orc_fractal *f, int64_t x, int64_t y) {
    if (x < 0 || y < 0 || x >= f->n || y >= f->n) return 0;
    for (int64_t mu = 0; mu < f->r; ++mu) {
        int64_t a = x % f->s, b = y % f->s;
        if (f->id[a + f->s * b] < 0) return 0;
        x /= f->s;
        y /= f->s;
    }
    return 1;
}

/* lambda: compact index -> embedded coordinate (digits of i in base k pick the
 * replica offset at each level, scaled by s^level). */
void orc_lambda(const orc_fractal *f, int64_t i, int64_t *x, int64_t *y) {
    int64_t px = 0, py = 0, scale = 1;
    for (int64_t mu = 0; mu < f->r; ++mu) {
        int64_t d = i % f->k;
        i /= f->k;
        px += f->ox[d] * scale;
        py += f->oy[d] * scale;
        scale *= f->s;
    }
    *x = px;
    *y = py;
}

/* nu: embedded coordinate -> compact index, or ORC_OUTSIDE. */
int64_t orc_nu(const orc_fractal *f, int64_t x, int64_t y) {
    if (x < 0 || y < 0 || x >= f->n || y >= f->n) return ORC_OUTSIDE;
    int64_t idx = 0, weight = 1;
    for (int64_t mu = 0; mu < f->r; ++mu) {
        int64_t a = x % f->s, b = y % f->s;
        int64_t h = f->id[a + f->s * b];
        if (h < 0) return ORC_OUTSIDE;
        idx += h * weight;
        weight *= f->k;
        x /= f->s;
        y /= f->s;
    }
    return idx;
}

/* The paper's 2D compact coordinate, eqs. (6)-(8):
 *   nu_x = sum_mu tau_x(k,mu) H(x,y,mu),  nu_y = sum_mu tau_y(k,mu) H(x,y,mu)
 * with tau_x = k^floor(mu/2) * ((mu+1) mod 2), tau_y = k^floor(mu/2) * (mu mod 2)
 * (eqs. 4-5).  Returns 0 and leaves the outputs unset for a non-member. */
int orc_nu_paper2d(const orc_fractal *f, int64_t x, int64_t y, int64_t *nx, int64_t *ny) {
    if (!orc_member(f, x, y)) return 0;
    int64_t sx = 0, sy = 0;
    for (int64_t mu = 0; mu < f->r; ++mu) {
        int64_t a = x % f->s, b = y % f->s;
        int64_t h = f->id[a + f->s * b];
        int64_t tk = ipow(f->k, mu / 2);
        int64_t tau_x = tk * ((mu + 1) % 2);
        int64_t tau_y = tk * (mu % 2);
        sx += tau_x * h;
        sy += tau_y * h;
        x /= f->s;
        y /= f->s;
    }
    *nx = sx;
    *ny = sy;
    return 1;
}

/* SplitMix64 (Steele, Lea & Flood 2014): the key-th output after seeding is
 * the mix of seed + (key+1) * gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t key) {
    const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
    uint64_t z = seed + (key + 1) * gamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* floor(p * 2^24) for p in [0,1]; both sides of the comparison use integers. */
uint32_t orc_threshold(double p) {
    if (!(p >= 0.0)) return 0;
    if (p >= 1.0) return 1u << 24;
    return (uint32_t)(p * 16777216.0);
}

static int orc_alive_at(const orc_fractal *f, int64_t x, int64_t y, uint64_t seed, uint32_t thr) {
    if (!orc_member(f, x, y)) return 0;
    uint64_t key = (uint64_t)y * (uint64_t)f->n + (uint64_t)x;
    return (orc_splitmix64(seed, key) >> 40) < thr;
}

/* Initial state on the n x n box (row-major, y*n + x). */
void orc_init_bbox(const orc_fractal *f, uint8_t *state, uint64_t seed, double p) {
    uint32_t thr = orc_threshold(p);
    int64_t n = f->n;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            state[y * n + x] = (uint8_t)orc_alive_at(f, x, y, seed, thr);
}

/* Initial state in compact order: cell i takes the value of lambda(i). */
void orc_init_compact(const orc_fractal *f, uint8_t *state, uint64_t seed, double p) {
    uint32_t thr = orc_threshold(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < f->cells; ++i) {
        int64_t x, y;
        orc_lambda(f, i, &x, &y);
        state[i] = (uint8_t)orc_alive_at(f, x, y, seed, thr);
    }
}

/* 1 for every member of the n x n box, 0 elsewhere. */
void orc_member_mask(const orc_fractal *f, uint8_t *mask) {
    int64_t n = f->n;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x) mask[y * n + x] = (uint8_t)orc_member(f, x, y);
}

static uint8_t orc_apply_rule(uint32_t rule, int64_t live_neighbours, int self_alive) {
    int64_t bit = live_neighbours + (self_alive ? 16 : 0);
    return (uint8_t)((rule >> bit) & 1u);
}

/* Whether the cell at offset (dx, dy) is a neighbour: the eight cells of the
 * Moore neighbourhood, or with bit 31 of the rule word only the four that
 * share an edge (section 3's example stencil). */
static int orc_neighbour(uint32_t rule, int64_t dx, int64_t dy) {
    if (dx == 0 && dy == 0) return 0;
    if ((rule >> 31) && dx != 0 && dy != 0) return 0;
    return 1;
}

/* One generation on the box.  mask is orc_member_mask's output; only member
 * neighbours inside the box count; non-members come out dead. */
void orc_bbox_step(const orc_fractal *f, const uint8_t *mask, const uint8_t *in, uint8_t *out,
                   uint32_t rule) {
    int64_t n = f->n;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y) {
        for (int64_t x = 0; x < n; ++x) {
            if (!mask[y * n + x]) {
                out[y * n + x] = 0;
                continue;
            }
            int64_t live = 0;
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    if (!orc_neighbour(rule, dx, dy)) continue;
                    int64_t xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= n || yy >= n) continue;
                    if (mask[yy * n + xx] && in[yy * n + xx]) ++live;
                }
            out[y * n + x] = orc_apply_rule(rule, live, in[y * n + x] != 0);
        }
    }
}

/* One generation in compact space, the paper's stencil procedure (section 3):
 * each compact cell finds its embedded coordinate with lambda, forms the
 * coordinates of its eight neighbours, maps each back with nu and reads it. */
void orc_compact_step(const orc_fractal *f, const uint8_t *in, uint8_t *out, uint32_t rule) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < f->cells; ++i) {
        int64_t x, y;
        orc_lambda(f, i, &x, &y);
        int64_t live = 0;
        for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
                if (!orc_neighbour(rule, dx, dy)) continue;
                int64_t j = orc_nu(f, x + dx, y + dy);
                if (j != ORC_OUTSIDE && in[j]) ++live;
            }
        out[i] = orc_apply_rule(rule, live, in[i] != 0);
    }
}

/* State of compact cell i after `steps` generations, from the state `in`,
 * by the definition itself: recursion over the cell's light cone (9^steps
 * evaluations).  For spot checks of large runs at small step counts. */
static uint8_t orc_cell_after(const orc_fractal *f, const uint8_t *in, int64_t i, uint32_t rule, int steps) {
    if (steps == 0) return in[i];
    int64_t x, y;
    orc_lambda(f, i, &x, &y);
    int64_t live = 0;
    for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
            if (!orc_neighbour(rule, dx, dy)) continue;
            int64_t j = orc_nu(f, x + dx, y + dy);
            if (j != ORC_OUTSIDE && orc_cell_after(f, in, j, rule, steps - 1)) ++live;
        }
    return orc_apply_rule(rule, live, orc_cell_after(f, in, i, rule, steps - 1) != 0);
}

void orc_cells_after(const orc_fractal *f, const uint8_t *in, const int64_t *idx, int64_t count,
                     uint32_t rule, int steps, uint8_t *out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) out[t] = orc_cell_after(f, in, idx[t], rule, steps);
}

/* The same light cone with the initial state of each cell taken from its
 * definition (member, SplitMix64 key y*n + x below the threshold) instead of
 * an array: for levels whose whole state is too large to build on the host. */
static uint8_t orc_cell_after_seeded(const orc_fractal *f, uint64_t seed, uint32_t thr, int64_t i, uint32_t rule,
                                     int steps) {
    int64_t x, y;
    orc_lambda(f, i, &x, &y);
    if (steps == 0) return (uint8_t)orc_alive_at(f, x, y, seed, thr);
    int64_t live = 0;
    for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
            if (!orc_neighbour(rule, dx, dy)) continue;
            int64_t j = orc_nu(f, x + dx, y + dy);
            if (j != ORC_OUTSIDE && orc_cell_after_seeded(f, seed, thr, j, rule, steps - 1)) ++live;
        }
    return orc_apply_rule(rule, live, orc_cell_after_seeded(f, seed, thr, i, rule, steps - 1) != 0);
}

void orc_cells_after_seeded(const orc_fractal *f, uint64_t seed, double p, const int64_t *idx, int64_t count,
                            uint32_t rule, int steps, uint8_t *out) {
    uint32_t thr = orc_threshold(p);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) out[t] = orc_cell_after_seeded(f, seed, thr, idx[t], rule, steps);
}

/* compact[i] = bbox[lambda(i)] */
void orc_gather(const orc_fractal *f, const uint8_t *bbox, uint8_t *compact) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < f->cells; ++i) {
        int64_t x, y;
        orc_lambda(f, i, &x, &y);
        compact[i] = bbox[y * f->n + x];
    }
}

/* bbox[lambda(i)] = compact[i]; every non-member cell becomes 0. */
void orc_expand(const orc_fractal *f, const uint8_t *compact, uint8_t *bbox) {
    memset(bbox, 0, (size_t)(f->n * f->n));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < f->cells; ++i) {
        int64_t x, y;
        orc_lambda(f, i, &x, &y);
        bbox[y * f->n + x] = compact[i];
    }
}

/* Vectorised forms of the maps, for the tests. */
void orc_lambda_many(const orc_fractal *f, const int64_t *idx, int64_t count, int64_t *x, int64_t *y) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) orc_lambda(f, idx[t], &x[t], &y[t]);
}

void orc_nu_many(const orc_fractal *f, const int64_t *x, const int64_t *y, int64_t count, int64_t *idx) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) idx[t] = orc_nu(f, x[t], y[t]);
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
