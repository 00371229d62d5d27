/*
 * libnbbfrac -- cellular-automaton steps on NBB fractals held in compact form,
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Quezada & Navarro, "Accelerating Compact Fractals with Tensor Core
 * GPUs" (technical report, 2021).  An NBB fractal F^{k,s} (section 1) at scale
 * level r lives in an n x n box, n = s^r, and has k^r cells (eq. 1).  Its
 * compact form stores only those k^r cells.  Two maps connect the spaces
 * (section 3): lambda takes a compact index to its (x, y) in the box, nu takes
 * (x, y) back to a compact index, or reports that the point is outside the
 * fractal.  A stencil step in compact space (section 3, last two paragraphs)
 * maps each cell with lambda, forms its neighbours' coordinates, maps them
 * back with nu and applies the update rule.
 *
 * Conventions used by every entry point
 *   - Coordinates: x to the right, y downwards, origin top-left (section 3).
 *   - Replica offsets: k pairs (x_j, y_j) in [0,s)^2, listed as
 *     x0,y0,x1,y1,...; list position j is replica id j, the value the helper H
 *     of section 3.1 returns for that digit pair.
 *   - Compact index: i = sum_{mu<r} H_mu k^mu, H_mu the replica id of the
 *     level-mu base-s digit pair of (x, y).  lambda(i) = sum_mu o_{d_mu(i)} s^mu
 *     with d_mu(i) the base-k digits of i.  (The paper draws the compact space
 *     as a 2D unfolding, eqs. 3-8; that is a fixed permutation of these
 *     indices.)  Every aligned run of k^m indices is then one level-m copy of
 *     the fractal.
 *   - State: one byte per cell, 0 = dead, 1 = alive.  Compact state is
 *     uint8[k^r] in compact-index order.  Box state is n rows of `pitch`
 *     bytes (cell (x,y) at y*pitch + x); pitch >= n and pitch % 16 == 0,
 *     nbb_bbox_pitch() gives the smallest one.  Cells of the box outside the
 *     fractal, and the padding columns x >= n, hold 0.
 *   - Rule word: bit c (c = 0..8) set = a dead cell with c live Moore
 *     neighbours is born; bit 16+c set = a live cell with c live neighbours
 *     survives; bit 31 (NBB_RULE_VON_NEUMANN) = count the four edge
 *     neighbours only.  Conway's Life B3/S23 is NBB_RULE_B3S23.  Cells
 *     outside the fractal or the box count as dead and stay dead.
 *   - Device pointers are owned by the caller and must be device memory of the
 *     device that was current at nbb_create (e.g. torch CUDA tensors).  A
 *     `stream` is a hipStream_t (NULL = the null stream).  Calls check their
 *     arguments, enqueue work and return; they do not wait for the device.
 *     Faults of the enqueued work surface at the next synchronisation.
 *   - Errors: every call returns an nbb_status; nbb_last_error() gives a
 *     message for the calling thread's last failure.  No exception crosses
 *     this interface.  A descriptor may be used from several threads at once
 *     except during nbb_configure and nbb_destroy.
 */
#ifndef NBBFRAC_H
#define NBBFRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NBB_OK = 0,
    NBB_E_INVALID = 1, /* bad argument: null pointer, wrong length, overlap, ... */
    NBB_E_RANGE = 2,   /* size beyond what the index types hold */
    NBB_E_NOMEM = 3,   /* device or host allocation failed */
    NBB_E_DEVICE = 4   /* HIP runtime error (no device, launch failure, ...) */
} nbb_status;

/* nu's result for a coordinate outside the box or outside the fractal. */
#define NBB_OUTSIDE 0xFFFFFFFFu

/* B3/S23: born with 3, survives with 2 or 3. */
#define NBB_RULE_B3S23 ((1u << 3) | ((1u << 2 | 1u << 3) << 16))

/* Rule-word flag: count only the four neighbours that share an edge with the
 * cell (the four-cell stencil of section 3's example) instead of the eight of
 * the Moore neighbourhood; counts then run 0..4. */
#define NBB_RULE_VON_NEUMANN (1u << 31)

/* How nbb_step_compact evaluates a step (nbb_configure). */
#define NBB_STRATEGY_AUTO 0u   /* TILED when the fractal allows it, else DIRECT */
#define NBB_STRATEGY_TILED 1u  /* level-m tiles staged in LDS with their halo */
#define NBB_STRATEGY_DIRECT 2u /* one thread per cell: lambda, 8 x nu, rule */
#define NBB_STRATEGY_TILED_WAVE 3u /* TILED with one wavefront per tile: for small tiles */
#define NBB_STRATEGY_TILED_BOX 4u  /* TILED, always in the byte-scatter form (see nbb_info.tiled_form) */
#define NBB_STRATEGY_TEMPORAL 5u   /* several generations per launch in LDS (small instances; nbb_configure_temporal) */
#define NBB_STRATEGY_TILED_EDGE 6u /* TILED, always in the edge-record form (NBB_E_INVALID where it does not apply) */

typedef struct nbb_fractal nbb_fractal;

typedef struct {
    uint64_t n;            /* box side s^r */
    uint64_t cells;        /* k^r */
    uint64_t tiles;        /* k^(r - tile_level) */
    uint32_t k, s, r;
    uint32_t strategy;     /* NBB_STRATEGY_TILED, _TILED_WAVE, _TEMPORAL or _DIRECT */
    uint32_t tile_level;   /* m: a tile is an aligned run of k^m compact cells */
    uint32_t tile_side;    /* s^m */
    uint32_t halo_cells;   /* neighbour cells staged per tile */
    uint32_t lds_bytes;    /* LDS used by one work-group of the tiled step */
    uint64_t bbox_pitch;   /* smallest pitch the box entry points accept */
    uint64_t device_table_bytes;
    /* Membership in the box entry points: the low L levels as an SL x SL
     * bitmap (SL = s^L <= 1024), the other r - L levels as an NH x NH byte
     * map (NH = s^(r-L)); a 16-column group of the box step can span two
     * high-level squares when SL is not a multiple of 16. */
    uint32_t box_low_side;  /* SL */
    uint32_t box_high_side; /* NH (0 when the box is too large to exist) */
    /* How a tiled strategy runs the step: 1 = edge records (each block's
     * cells loaded into registers, only the blocks' edge rows and columns
     * exchanged through LDS; TILED_EDGE, and TILED where the level allows
     * the form and its blocks fill at least three quarters of the work-group
     * passes over them), 2 = byte scatter (the tile's cells scattered into
     * an LDS box: TILED elsewhere, TILED_BOX, TILED_WAVE); 3 = TEMPORAL;
     * 0 for DIRECT. */
    uint32_t tiled_form;
    uint32_t temporal_depth; /* TEMPORAL: ring depth h = generations per launch at most; else 0 */
} nbb_info;

/*
 * Create the descriptor of F^{k,s} at level r (sections 1 and 3.1) and upload
 * its tables to the current device.
 *   offsets: 2k int32 values x0,y0,...; each pair in [0,s)^2, no duplicates.
 * Returns NBB_E_INVALID for out == NULL, offsets == NULL, k == 0, s < 2,
 * s > 16, k > s*s, an offset outside [0,s)^2 or a repeated offset;
 * NBB_E_RANGE if k^r > 2^32 - 1 or s^r + 1 > 2^31 - 1; NBB_E_DEVICE /
 * NBB_E_NOMEM if the tables cannot be uploaded.  On failure *out is NULL.
 * The descriptor owns its host and device tables; free with nbb_destroy.
 */
nbb_status nbb_create(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r,
                      nbb_fractal **out);

/* Free a descriptor (NULL is a no-op).  No enqueued work may still use it. */
void nbb_destroy(nbb_fractal *f);

/* Describe a descriptor.  NBB_E_INVALID for NULL arguments. */
nbb_status nbb_query(const nbb_fractal *f, nbb_info *info);

/*
 * Choose how nbb_step_compact runs: strategy NBB_STRATEGY_* and, for TILED,
 * TILED_BOX and TILED_WAVE, the tile level m (0 = automatic; otherwise
 * 1 <= m <= r).  TILED_BOX is TILED held to the byte-scatter form, TILED_EDGE
 * TILED held to the edge-record form (nbb_query then reports strategy TILED
 * with tiled_form 2 or 1; TILED_EDGE fails where the form does not apply:
 * blocks of side other than 3 or 4, tiles below two loads' width, more than
 * 1024 blocks or 512 halo blocks, a record grid beyond 64 KiB).
 * Both need 2 <= s <= 4 and r >= 1; TILED_WAVE also needs a tile small
 * enough for one wavefront (k^m + 30 <= 2048 cells, at most 256 halo cells
 * and blocks, four LDS boxes within 64 KiB).  NBB_E_INVALID when the request
 * cannot be met (the descriptor keeps its previous plan).  Rebuilds and re-uploads the tile
 * tables; must not overlap other calls on the same descriptor, and no
 * enqueued work may still use the old tables (synchronise first).  The
 * packed step's 32-phase table follows the new plan at its next call, with
 * the same condition.
 */
nbb_status nbb_configure(nbb_fractal *f, uint32_t strategy, uint32_t tile_level);

/*
 * Several generations per launch (temporal blocking over section 3's
 * blocked approach), for instances too small to fill the GPU: work-group t
 * holds tile t (k^m compact cells, the S x S square of one level-m copy,
 * S = s^m) and every cell of its eight neighbour tiles within distance h
 * (`depth`) of the square as a box of side S + 2h in LDS, applies up to h
 * generations to the whole box there and stores the tile's own cells; a
 * generation on the box is exact wherever its 3 x 3 neighbourhood was, so
 * the tile stays exact for h generations.  nbb_step_compact then runs
 * ceil(steps / h) launches (one more when needed so that the result still
 * ends in b iff steps is odd), each of up to h generations.  tile_level and
 * depth 0 choose automatically (h = min(16, S); the level, among those with
 * S <= 81, with the least estimated time per generation from a launch cost
 * per h generations, a cost per wave of tiles over the CUs and the box's
 * cells).  The
 * box, its copy and a member mask (3 (S+2h) ceil4(S+2h) bytes) must fit one
 * work-group's LDS.  Needs 2 <= s <= 4; 1 <= tile_level <= r and
 * 1 <= depth <= S when given.  NBB_E_INVALID otherwise (the descriptor keeps
 * its plan).  nbb_query reports strategy NBB_STRATEGY_TEMPORAL, the level,
 * tiles, ring cells (halo_cells), LDS and temporal_depth; batches step the
 * descriptor with its tile plan as before.  Same conditions as
 * nbb_configure for work in flight.
 */
nbb_status nbb_configure_temporal(nbb_fractal *f, uint32_t tile_level, uint32_t depth);

/*
 * lambda (section 3): x[t], y[t] = embedded coordinate of compact index idx[t],
 * t < count.  idx == NULL means idx[t] = t.  An index >= k^r gives x = y = -1.
 * Device arrays; count == 0 is a no-op.
 */
nbb_status nbb_lambda(const nbb_fractal *f, const uint32_t *idx, uint64_t count, int32_t *x,
                      int32_t *y, void *stream);

/*
 * nu (section 3.1, eqs. 6-8 in compact-index form): idx[t] = compact index of
 * (x[t], y[t]), or NBB_OUTSIDE when the point is outside [0,n)^2 or not a
 * fractal cell.  Device arrays; count == 0 is a no-op.
 */
nbb_status nbb_nu(const nbb_fractal *f, const int32_t *x, const int32_t *y, uint64_t count,
                  uint32_t *idx, void *stream);

/*
 * The same maps evaluated three ways (results identical):
 *   NBB_MAP_LUT    chunked look-up tables (the default of nbb_lambda / nbb_nu,
 *                  and the fastest form on gfx950);
 *   NBB_MAP_DIGITS one level per step, as the per-thread maps of section 3.1;
 *   NBB_MAP_MFMA   measurement only (about ten times slower than
 *                  NBB_MAP_LUT on MI355X, kept to compare against the
 *                  paper's matrix-unit form, never chosen by any other call):
 *                  digits per item as NBB_MAP_DIGITS, the per-level sum as
 *                  an int8 matrix-core contraction (the matrix encoding of
 *                  section 3.1 on gfx950 matrix cores: one-hot digits, resp.
 *                  replica ids, times 7-bit planes of o_j s^mu, resp. j k^mu;
 *                  needs r*k <= 192 and n <= 2^28, else NBB_E_INVALID).
 * Same arguments, results and errors as nbb_lambda / nbb_nu otherwise.
 */
#define NBB_MAP_LUT 0u
#define NBB_MAP_DIGITS 1u
#define NBB_MAP_MFMA 2u
nbb_status nbb_lambda_method(const nbb_fractal *f, uint32_t method, const uint32_t *idx, uint64_t count,
                             int32_t *x, int32_t *y, void *stream);
nbb_status nbb_nu_method(const nbb_fractal *f, uint32_t method, const int32_t *x, const int32_t *y,
                         uint64_t count, uint32_t *idx, void *stream);

/*
 * Bernoulli(p) initial state.  Cell (x, y) of the fractal is alive iff the top
 * 24 bits of SplitMix64 output number key = y*n + x of the stream seeded with
 * `seed` (Steele, Lea & Flood 2014: mix(seed + (key+1)*0x9E3779B97F4A7C15))
 * are below floor(p * 2^24).  Both layouts therefore hold the same state.
 * nbb_init_compact: len must be k^r.  nbb_init_bbox: len must be n*pitch,
 * pitch as described above; non-members and padding are written 0.
 * p must lie in [0, 1].  The state buffer must be 16-byte aligned
 * (NBB_E_INVALID otherwise): the kernels write 16 cells per store.
 */
nbb_status nbb_init_compact(const nbb_fractal *f, uint8_t *state, uint64_t len, uint64_t seed,
                            double p, void *stream);
nbb_status nbb_init_bbox(const nbb_fractal *f, uint8_t *state, uint64_t pitch, uint64_t len,
                         uint64_t seed, double p, void *stream);

/*
 * `steps` synchronous generations of `rule` on the compact state (section 3,
 * stencil procedure; section 4, Game of Life on the fractal).  The state
 * starts in a; buffers a and b alternate, and *result_in_b (if not NULL) is
 * set to steps & 1, i.e. whether the result ended in b.  len must be k^r;
 * a and b must not overlap and must both be 16-byte aligned (the tiled step
 * reads 16-byte chunks); the rule may only use bits 0-8, 16-24 and 31; state
 * bytes must be 0 or 1.  steps == 0 leaves both buffers untouched.
 * NBB_E_INVALID for a violation of any of these.
 */
nbb_status nbb_step_compact(const nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t len,
                            uint32_t steps, uint32_t rule, int *result_in_b, void *stream);

/*
 * The bounding-box baseline the paper compares against (section 4, method 1):
 * the same generations computed on the whole box, every box cell visited.
 * len must be n*pitch; a and b must be 16-byte aligned (rows are read and
 * written 16 bytes at a time) and must not overlap.  The input must hold 0
 * at non-members and padding; the output does too.  Other rules as
 * nbb_step_compact.
 */
nbb_status nbb_step_bbox(const nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t pitch,
                         uint64_t len, uint32_t steps, uint32_t rule, int *result_in_b,
                         void *stream);

/*
 * The paper's lambda approach (section 4, second method): the same
 * generations on the box layout, but with one thread per fractal cell, which
 * finds its box position with lambda and reads its neighbours from the box
 * directly.  Arguments, result buffer, alignment and errors as
 * nbb_step_bbox; the input must hold 0 at non-members and padding, and b is
 * cleared once per call
 * (steps >= 1) so that its non-members hold 0 too.
 */
nbb_status nbb_step_lambda(const nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t pitch,
                           uint64_t len, uint32_t steps, uint32_t rule, int *result_in_b,
                           void *stream);

/*
 * Blocked layout (section 3, blocked approach: the compact space as a packed
 * collection of small bounding boxes, one per coarse cell).  With the
 * descriptor's tiled plan at tile level m (S = s^m, k^(r-m) tiles), tile t is
 * stored as its whole S x S square at bytes [t S^2, (t+1) S^2): cell (x, y)
 * of the square at t S^2 + y S + x, positions outside the fractal 0.  Memory
 * is (s^2/k)^m times the compact size; steps touch every position of every
 * square.  Needs a TILED or TILED_WAVE plan (NBB_E_INVALID otherwise); the
 * layout follows the plan, so nbb_configure changes it.
 *   nbb_blocked_bytes: k^(r-m) S^2 (0 without a tiled plan).
 *   nbb_blocked_from_compact / _to_compact: conversions; len is the blocked
 *   length, the compact side is k^r bytes; blocked buffers 16-byte aligned.
 *   nbb_step_blocked: generations on the blocked layout, arguments and
 *   result buffer as nbb_step_compact (the input must hold 0 at
 *   non-members; the output does too).
 */
uint64_t nbb_blocked_bytes(const nbb_fractal *f);
nbb_status nbb_blocked_from_compact(const nbb_fractal *f, const uint8_t *compact, uint8_t *blocked,
                                    uint64_t len, void *stream);
nbb_status nbb_blocked_to_compact(const nbb_fractal *f, const uint8_t *blocked, uint64_t len,
                                  uint8_t *compact, void *stream);
nbb_status nbb_step_blocked(const nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                            uint32_t rule, int *result_in_b, void *stream);

/*
 * Bit-packed compact state (the byte layout at one bit per cell, 8x fewer
 * bytes): a capacity form, for states that would not fit as bytes.  Its step
 * scatters the bits into the byte step's LDS box and runs the byte rule, so it
 * is slower than the byte step (triangle r16: 49 us per generation against
 * 25-28); it does not cut the step's time.  Cell i is bit i % 32 of the
 * little-endian 32-bit word i / 32, i.e. bit i % 8 of byte i / 8.  Needs a
 * TILED or TILED_WAVE plan (NBB_E_INVALID otherwise).
 *   nbb_packed_bytes: 4 ceil(k^r / 32) (0 for NULL).  Bits past the last cell
 *   are 0 after nbb_pack and are never written by nbb_step_packed.
 *   nbb_pack: packed = bits of compact (k^r bytes; any non-zero byte packs as
 *   1).  nbb_unpack: compact (k^r bytes, 0 or 1) from packed.  len is the
 *   packed length, which must equal nbb_packed_bytes; packed buffers 4-byte
 *   aligned.
 *   nbb_step_packed: generations on packed states, arguments and result
 *   buffer as nbb_step_compact (a and b packed, len = nbb_packed_bytes).
 *   The descriptor's tile plan is used (after nbb_configure, the new one);
 *   NBB_E_INVALID if a tile's output words do not fit the kernel's limits
 *   (at most 1024 blocks, 1024 halo cells and 16 cells per block: every
 *   automatic plan fits).  The first call for a plan builds a 32-phase copy
 *   of its scatter table on the device (kept with the descriptor).
 */
uint64_t nbb_packed_bytes(const nbb_fractal *f);
nbb_status nbb_pack(const nbb_fractal *f, const uint8_t *compact, uint8_t *packed, uint64_t len, void *stream);
nbb_status nbb_unpack(const nbb_fractal *f, const uint8_t *packed, uint64_t len, uint8_t *compact, void *stream);
nbb_status nbb_step_packed(const nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                           uint32_t rule, int *result_in_b, void *stream);

/* bbox[lambda(i)] = compact[i]; every other box byte becomes 0. */
nbb_status nbb_expand(const nbb_fractal *f, const uint8_t *compact, uint8_t *bbox, uint64_t pitch,
                      uint64_t len, void *stream);

/* compact[i] = bbox[lambda(i)] (the inverse of nbb_expand on members). */
nbb_status nbb_gather(const nbb_fractal *f, const uint8_t *bbox, uint64_t pitch, uint8_t *compact,
                      uint64_t len, void *stream);

/*
 * Autotuner.  The paper picks its block size per method by measurement
 * (section 4: the best rho differs between methods); this does the same for
 * the compact step.  Times `steps` generations (after one untimed one) of
 * each candidate -- TILED_EDGE, TILED_BOX and TILED_WAVE at every tile level
 * m whose tile holds at least 128 cells, plus the largest level that fits;
 * when steps > 1, TEMPORAL at its automatic plan and at every level of side
 * <= 81 with ring depths 8 and 16; and DIRECT -- on the caller's
 * buffers a and b (their contents are overwritten: pass a copy of a
 * representative state), then configures the fastest, as nbb_configure would.
 * Waits for `stream`.  Arguments as nbb_step_compact (a and b 16-byte
 * aligned, not overlapping); steps >= 1.  If info is
 * not NULL it receives nbb_query's result for the chosen plan.  Must not
 * overlap other calls on the same descriptor.
 */
nbb_status nbb_autotune(nbb_fractal *f, uint8_t *a, uint8_t *b, uint64_t len, uint32_t steps,
                        uint32_t rule, void *stream, nbb_info *info);

/*
 * Batches: many independent automata, each on a fractal of its own (own k, s,
 * offsets and r), stepped together.  All states live in one device arena per
 * buffer: instance i occupies bytes [offsets[i], offsets[i] + k_i^r_i) of
 * both arenas passed to nbb_batch_step.  Instances whose descriptors use the
 * same tiled strategy at the same tile level for the same (k, s, offsets) form one
 * group and are stepped by one launch per generation over all their tiles
 * (configure a common tile level with nbb_configure to group instances of
 * different r); instances with the DIRECT strategy are stepped one launch
 * each.  Small tiled instances, those whose state fits one work-group's LDS
 * twice over, with the tile boxes and the neighbour table (160 KiB on gfx950;
 * e.g. up to 3^9 triangle or 7^5 H cells), and whose generation takes at most
 * 8 passes of up to 4 tiles, may instead be stepped in LDS (by default when
 * they hold at least 1/8 of the batch's tiled cells; see
 * nbb_batch_create_ex): one work-group per instance runs all of the call's
 * generations of it in one launch, with no global traffic between
 * generations, at a tile level of its own (the one with the fewest passes;
 * built with the descriptor on the first batch that needs it, and independent
 * of nbb_configure).  All of them share one launch; beside group or direct
 * launches it runs on a side stream of the library (one per device, kept
 * until the process ends) that is forked from `stream` at the start of each
 * step call and joined back to it before the call's last enqueued work (so,
 * seen from `stream`, the call's work is ordered as before).  With more than
 * one group, groups after the first run on up to three more streams of the
 * library (per device, kept until the process ends), forked and joined the
 * same way, so that one group's launches fill the start and the end of
 * another's; the batch built by nbb_batch_step_each_noalloc runs every group
 * on `stream`.  Step calls on one batch
 * share its small device tables: enqueue them from one host thread, and order
 * calls made on different streams (an event) before the later one starts.
 *
 * nbb_batch_create: fractals[i] (may repeat) must outlive the batch and keep
 * their configuration while it exists; offsets[i] must be multiples of 16,
 * the ranges must not overlap, and every offset must be below 2^36.  Builds
 * the batch's tile tables on the current device (the descriptors' device)
 * with work enqueued on `stream`.  count == 0 gives an empty batch.
 * NBB_E_INVALID for NULL pointers, a descriptor of another device, misaligned
 * or overlapping ranges; NBB_E_RANGE beyond the limits above or 2^28 tiles in
 * one group.  Free with nbb_batch_destroy (no enqueued work may still use it).
 */
typedef struct nbb_batch nbb_batch;
typedef struct {
    uint32_t instances;
    uint32_t groups;          /* one launch per generation each */
    uint32_t direct;          /* instances stepped by their own launch */
    uint32_t resident;        /* instances stepped in LDS, all generations in one launch */
    uint64_t cells;           /* sum of k_i^r_i */
    uint64_t tiles;           /* tiles of all tiled instances (groups and resident) */
    uint64_t arena_bytes;     /* smallest arena: max(offset + cells) rounded up to 16 */
    uint64_t device_table_bytes;
} nbb_batch_info;
nbb_status nbb_batch_create(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                            void *stream, nbb_batch **out);
/* As nbb_batch_create (flags 0: the default choice above), with flags:
 * NBB_BATCH_NO_RESIDENT steps every tiled instance by the per-generation group
 * launches, small ones included; NBB_BATCH_RESIDENT steps every small one in
 * LDS, whatever its share of the cells.  NBB_E_INVALID for unknown flag bits
 * or both flags. */
#define NBB_BATCH_NO_RESIDENT 1u
#define NBB_BATCH_RESIDENT 2u
nbb_status nbb_batch_create_ex(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                               uint32_t flags, void *stream, nbb_batch **out);
void nbb_batch_destroy(nbb_batch *batch);
nbb_status nbb_batch_query(const nbb_batch *batch, nbb_batch_info *info);

/*
 * `steps` generations of `rule` for every instance of the batch, states
 * starting in arena a, alternating with arena b as nbb_step_compact does
 * (*result_in_b = steps & 1).  Both arenas must be 16-byte aligned, at least
 * arena_bytes long (arena_len), and must not overlap; bytes outside the
 * instances' ranges are not written (loads of a block may reach past its
 * instance's range, never past arena_len; those bytes are not used).  Only
 * the result is
 * specified: an instance's range in the other arena holds some earlier
 * generation (instances stepped in LDS leave it untouched).
 */
nbb_status nbb_batch_step(const nbb_batch *batch, uint8_t *a, uint8_t *b, uint64_t arena_len, uint32_t steps,
                          uint32_t rule, int *result_in_b, void *stream);

/*
 * As nbb_batch_step, but instance i (numbered as in nbb_batch_create) takes
 * steps[i] generations: generation g runs only the instances with
 * steps[i] > g, so instance i's result ends in b iff steps[i] is odd and an
 * instance with 0 steps is left untouched.  Within each group the step
 * counts must not increase in the order the instances were given to
 * nbb_batch_create (NBB_E_INVALID otherwise; instances stepped in LDS are
 * exempt): list instances by decreasing step count.  steps is a host array of
 * nbb_batch_info.instances entries.
 */
nbb_status nbb_batch_step_each(const nbb_batch *batch, uint8_t *a, uint8_t *b, uint64_t arena_len,
                               const uint32_t *steps, uint32_t rule, void *stream);

/*
 * Tile plans for a batch chosen by measurement (section 4 picks each
 * method's block size by timing it).  The instances are grouped by fractal
 * (k, s, offsets; fractals the tiled step does not support are left alone);
 * for each group every candidate plan that all its descriptors accept - the
 * tile levels up to the group's smallest r whose tiles hold at least 64
 * cells (and the largest level), each in the edge-record and in the
 * byte-scatter form - is timed on a batch of exactly the group's instances
 * (group launches, none in LDS) for `steps` generations after one warm-up
 * generation, and every descriptor of the group is configured to the
 * fastest.  Results are kept for the process, keyed by device, fractal, the
 * group's smallest and largest r and the rule's form (B3/S23, table rule,
 * any rule), and reused without timing unless flags has NBB_TUNE_NO_CACHE.
 * The states in a and b are stepped (their values are then unspecified);
 * arguments as nbb_batch_step_each_noalloc.  Synchronise work that uses the
 * descriptors before the call; it synchronises on `stream` itself.  Batches
 * built earlier from these descriptors must be rebuilt afterwards.
 */
#define NBB_TUNE_NO_CACHE 1u
nbb_status nbb_batch_autotune(nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count, uint8_t *a,
                              uint8_t *b, uint64_t arena_len, uint32_t steps, uint32_t rule, uint32_t flags,
                              void *stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Does what
 * nbb_batch_create_ex(fractals, offsets, count, NBB_BATCH_NO_RESIDENT, ...),
 * nbb_batch_step_each(..., steps, rule, stream) and nbb_batch_destroy do
 * together, with the same arguments, checks and results, but calls no
 * hipMalloc / hipFree and waits on nothing: the batch's tables (per instance
 * 24 bytes, per tile 40 bytes, each group's part rounded up to 256) are
 * rebuilt at every call, by kernels enqueued on `stream`, inside a static
 * device array of the library of NBB_NOALLOC_SCRATCH_BYTES (one per device,
 * held until the process ends).  Every instance goes through the
 * per-generation group launches (none is stepped in LDS).  NBB_E_RANGE if the
 * tables would exceed the array (about 400,000 tiles), before anything is
 * enqueued.  All calls on one device share the array and leave their tables
 * in it: calls enqueued on one stream are ordered and safe; calls that overlap
 * on one device (other streams, other host threads without an event between
 * them) race and give undefined results.  The descriptors must not be
 * reconfigured while their work is enqueued.
 */
#define NBB_NOALLOC_SCRATCH_BYTES (16u << 20)
nbb_status nbb_batch_step_each_noalloc(const nbb_fractal *const *fractals, const uint64_t *offsets, uint32_t count,
                                       uint8_t *a, uint8_t *b, uint64_t arena_len, const uint32_t *steps,
                                       uint32_t rule, void *stream);

/* Smallest box pitch for this descriptor: n rounded up to a multiple of 16. */
uint64_t nbb_bbox_pitch(const nbb_fractal *f);

/* Message for the calling thread's last failed call ("" if none). */
const char *nbb_last_error(void);

/* Name of a status code. */
const char *nbb_status_string(nbb_status s);

/*
 * Host-side view of the tile plan the tiled step would use for F^{k,s} at
 * level r with tile level m (0 = automatic), without touching a device.  For
 * inspection and tests.  The arrays belong to the plan; free it with
 * nbb_plan_free.
 *   lut0[i], i < tile_cells: byte offset in the tile's LDS box of local cell i
 *   lut1[b], b < blocks: offset of the window corner (one row up, one column
 *   left) of block b, a level-block_level square of side block_side
 *   The box has box_rows rows of box_pitch bytes; tile cell (x, y) sits at
 *   row y+1, column x+1.  Rows and columns that no block window reaches are
 *   left out (box_rows <= tile_side + 2).
 *   halo_src[h] = (direction << 29) | local index in that neighbour tile,
 *   direction = (dy+1)*3 + (dx+1) skipping the centre (0..7), for every cell
 *   of a neighbouring tile that lands inside the box;
 *   halo_dst[h] = byte offset in the LDS box;
 *   nbr[8 t + d] = tile in direction d of tile t (same numbering), or
 *   0xFFFFFFFF where that block of the box holds no fractal cell.
 *
 * The edge-record form at the same level (edge_ok = 0 where it does not
 * apply): blocks sit on an edge_grid x edge_grid grid (block b at
 * lambda_{m-q}(b) in block units) with a one-block ring for the halo items;
 * each has a record of 16 bytes: block b is record b, halo item h record
 * blocks + h, and the last of the edge_records records (edge_rec_bytes in
 * all, rounded up to 4 records) is all zeros, standing for positions with no
 * block.
 *   edge_blk[4b .. 4b+3] = the records of block b's neighbours, two per word
 *   (low half first): left | right, above | below, above-left | above-right,
 *   below-left | below-right (the step reads a block's bytes as edge_nsrc
 *   dwords through one aligned load of a window holding them);
 *   edge_halo[2h] = direction << 29 | block of that neighbour tile,
 *   edge_halo[2h+1] = its record, for edge_halo_count items;
 *   edge_unpack / edge_pack: the v_perm selectors from a block's bytes to its
 *   rows and from next-state rows back to compact order ([0..3] for rows or
 *   output dwords 0-3 from the first pair of sources, [4..7] from the second).
 */
typedef struct nbb_plan nbb_plan;
typedef struct {
    uint32_t tile_level, tile_side, tile_cells, block_level, block_side, blocks, halo_count;
    uint32_t box_pitch, box_rows, lds_bytes;
    uint64_t tiles;
    const uint16_t *lut0;
    const uint16_t *lut1;
    const uint32_t *halo_src;
    const uint32_t *halo_dst;
    const uint32_t *nbr;
    uint32_t edge_ok, edge_grid, edge_records, edge_rec_bytes, edge_halo_count, edge_nsrc;
    uint32_t edge_unpack[8], edge_pack[8];
    const uint32_t *edge_blk;
    const uint32_t *edge_halo;
} nbb_plan_view;
nbb_status nbb_plan_build(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r,
                          uint32_t tile_level, nbb_plan **out, nbb_plan_view *view);
void nbb_plan_free(nbb_plan *p);

/*
 * Host-side view of the temporal plan (nbb_configure_temporal) for F^{k,s}
 * at level r, tile level m and ring depth h (both explicit, >= 1), without a
 * device; lds_limit bytes for the three boxes (0: 160 KiB).  Box row y,
 * column x (pitch box_pitch bytes) is the embedded point (x - h, y - h)
 * relative to the tile's corner.
 *   self[j], j < tile_cells: box byte offset of local cell j
 *   halo[2e], halo[2e+1], e < halo_count: (direction << 29) | local index of
 *   a cell of neighbour tile `direction` (numbered as nbr below) that lies in
 *   the box, and its box byte offset
 *   nbr[8t + d]: neighbour tile d of tile t, d = (dy+1)*3 + (dx+1) skipping
 *   the centre, 0xFFFFFFFF where none
 * NBB_E_INVALID for bad arguments; free with nbb_temporal_plan_free.
 */
typedef struct nbb_temporal_plan nbb_temporal_plan;
typedef struct {
    uint32_t tile_level, tile_side, tile_cells, depth, box_side, box_pitch, lds_bytes, halo_count;
    uint64_t tiles;
    const uint32_t *self;
    const uint32_t *halo;
    const uint32_t *nbr;
} nbb_temporal_view;
nbb_status nbb_temporal_plan_build(uint32_t k, uint32_t s, const int32_t *offsets, uint32_t r, uint32_t tile_level,
                                   uint32_t depth, uint32_t lds_limit, nbb_temporal_plan **out,
                                   nbb_temporal_view *view);
void nbb_temporal_plan_free(nbb_temporal_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* NBBFRAC_H */
