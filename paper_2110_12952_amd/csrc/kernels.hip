// HIP kernels for gfx950 (MI355X): the maps lambda / nu, the compact-space
// automaton step (tiled and per-cell), the bounding-box step, and the
// initial-state / layout-conversion kernels.
//
// Wavefronts are 64 lanes.  State is one byte per cell; four cells share a
// dword and neighbour counts are formed four bytes at a time (SWAR): no count
// exceeds 9, so byte lanes never carry into each other.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "kernels.hpp"

#include "device_common.hpp"
#include "edges_launch.hpp"
#include "tiled_launch.hpp"

namespace nbb {

// ---------------------------------------------------------------------------
// lambda / nu, chunked look-up tables held in LDS (section 3: lambda maps
// compact -> embedded, nu embedded -> compact; section 3.1 builds nu from the
// per-level replica id H; both are sums of one term per level, here evaluated
// jl (resp. jn) levels per table look-up).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lam_lut(const MapParams &P, const uint32_t *lam, uint32_t i,
                                        uint32_t &x, uint32_t &y) {
    uint32_t px = 0, py = 0, scale = 1;
    for (uint32_t c = 0; c + 1 < P.nchunks_l; ++c) {
        uint32_t q = udiv(P.divkl, i);
        uint32_t e = lam[i - q * P.kl];
        px += (e & 0xFFFFu) * scale;
        py += (e >> 16) * scale;
        scale *= P.sl;
        i = q;
    }
    if (P.nchunks_l) {
        uint32_t e = lam[P.lam_top_off + i];
        px += (e & 0xFFFFu) * scale;
        py += (e >> 16) * scale;
    }
    x = px;
    y = py;
}

__device__ __forceinline__ uint32_t nu_lut(const MapParams &P, const uint16_t *nu, int32_t x,
                                           int32_t y) {
    if (uint32_t(x) >= P.n || uint32_t(y) >= P.n) return kOutside;
    uint32_t ux = uint32_t(x), uy = uint32_t(y), idx = 0, w = 1, bad = 0;
    for (uint32_t c = 0; c + 1 < P.nchunks_n; ++c) {
        uint32_t qx = udiv(P.divsn, ux), qy = udiv(P.divsn, uy);
        uint32_t v = nu[(uy - qy * P.sn) * P.sn + (ux - qx * P.sn)];
        bad |= (v == 0xFFFFu);
        idx += v * w;
        w *= P.kn;
        ux = qx;
        uy = qy;
    }
    if (P.nchunks_n) {
        uint32_t v = nu[P.nu_top_off + uy * P.sn_top + ux];
        bad |= (v == 0xFFFFu);
        idx += v * w;
    }
    return bad ? kOutside : idx;
}

// Cooperative copy of the map tables into LDS.  Layout: lambda table
// (lam_words u32) then nu table (nu_halves u16).
__device__ __forceinline__ void load_map_tables(const MapParams &P, uint32_t lam_words,
                                                uint32_t nu_halves, uint32_t *lam, uint16_t *nu) {
    for (uint32_t t = threadIdx.x; t < lam_words; t += blockDim.x) lam[t] = P.lam_lut[t];
    for (uint32_t t = threadIdx.x; t < nu_halves; t += blockDim.x) nu[t] = P.nu_lut[t];
    __syncthreads();
}

__global__ __launch_bounds__(512) void k_lambda(MapParams P, uint32_t lam_words,
                                                const uint32_t *__restrict__ idx, uint64_t count,
                                                int32_t *__restrict__ x, int32_t *__restrict__ y) {
    extern __shared__ __align__(16) uint32_t smem_l[];
    load_map_tables(P, lam_words, 0, smem_l, nullptr);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride) {
        uint64_t i = idx ? uint64_t(idx[t]) : t;
        int32_t ox = -1, oy = -1;
        if (i <= P.cells_m1) {
            uint32_t ux, uy;
            lam_lut(P, smem_l, uint32_t(i), ux, uy);
            ox = int32_t(ux);
            oy = int32_t(uy);
        }
        x[t] = ox;
        y[t] = oy;
    }
}

__global__ __launch_bounds__(512) void k_nu(MapParams P, uint32_t nu_halves,
                                            const int32_t *__restrict__ x,
                                            const int32_t *__restrict__ y, uint64_t count,
                                            uint32_t *__restrict__ idx) {
    extern __shared__ __align__(16) uint16_t smem_n[];
    load_map_tables(P, 0, nu_halves, nullptr, smem_n);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
        idx[t] = nu_lut(P, smem_n, x[t], y[t]);
}

// lambda with one digit per step, the paper's per-thread map (section 3.1,
// evaluated level by level): d_mu = i mod k, i /= k, x += o_{d_mu}.x s^mu.
__device__ __forceinline__ void lam_digits(const MapParams &P, const uint8_t *sox, const uint8_t *soy,
                                           uint32_t i, uint32_t &x, uint32_t &y) {
    uint32_t px = 0, py = 0, scale = 1;
    for (uint32_t mu = 0; mu < P.r; ++mu) {
        const uint32_t q = udiv(P.divk, i);
        const uint32_t d = i - q * P.k;
        px += sox[d] * scale;
        py += soy[d] * scale;
        scale *= P.s;
        i = q;
    }
    x = px;
    y = py;
}
// nu one level per step (eqs. 6-8 in compact-index form): the level-mu digit
// pair gives H_mu, idx += H_mu k^mu; any pair outside the offsets -> outside.
__device__ __forceinline__ uint32_t nu_digits(const MapParams &P, const uint8_t *shl, int32_t X, int32_t Y) {
    if (uint32_t(X) >= P.n || uint32_t(Y) >= P.n) return kOutside;
    uint32_t x = uint32_t(X), y = uint32_t(Y), idx = 0, w = 1, bad = 0;
    for (uint32_t mu = 0; mu < P.r; ++mu) {
        const uint32_t qx = udiv(P.divs, x), qy = udiv(P.divs, y);
        const uint32_t h = shl[(x - qx * P.s) + P.s * (y - qy * P.s)];
        bad |= (h == 0xFFu);
        idx += h * w;
        w *= P.k;
        x = qx;
        y = qy;
    }
    return bad ? kOutside : idx;
}

__device__ __forceinline__ void load_small_tables(const MapParams &P, uint8_t *sox, uint8_t *soy, uint8_t *shl) {
    for (uint32_t t = threadIdx.x; t < 256; t += blockDim.x) {
        sox[t] = t < P.k ? P.ox[t] : 0;
        soy[t] = t < P.k ? P.oy[t] : 0;
        shl[t] = P.hl[t];
    }
    __syncthreads();
}

__global__ __launch_bounds__(512) void k_lambda_digits(MapParams P, const uint32_t *__restrict__ idx,
                                                       uint64_t count, int32_t *__restrict__ x,
                                                       int32_t *__restrict__ y) {
    __shared__ uint8_t sox[256], soy[256], shl[256];
    load_small_tables(P, sox, soy, shl);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride) {
        const uint64_t i = idx ? uint64_t(idx[t]) : t;
        int32_t ox = -1, oy = -1;
        if (i <= P.cells_m1) {
            uint32_t ux, uy;
            lam_digits(P, sox, soy, uint32_t(i), ux, uy);
            ox = int32_t(ux);
            oy = int32_t(uy);
        }
        x[t] = ox;
        y[t] = oy;
    }
}

__global__ __launch_bounds__(512) void k_nu_digits(MapParams P, const int32_t *__restrict__ x,
                                                   const int32_t *__restrict__ y, uint64_t count,
                                                   uint32_t *__restrict__ idx) {
    __shared__ uint8_t sox[256], soy[256], shl[256];
    load_small_tables(P, sox, soy, shl);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
        idx[t] = nu_digits(P, shl, x[t], y[t]);
}

// lambda with the per-level sum on the matrix cores (v_mfma_i32_16x16x32_i8).
// Each lane takes one item, extracts its r digits (as k_lambda_digits) and
// writes their one-hot bytes, item-major, to LDS; each 16-item group is then
// one B operand (lane j + 16 q holds item j's K bytes 8q..8q+7 of a K tile),
// multiplied by the constant A.  In D, lanes 0-15 hold the x planes (rows
// 0-3) and lanes 16-31 the y planes (rows 4-7) of items 0-15.
typedef int v4i32 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_lambda_mfma(MapParams P, MfmaLambda M, const uint32_t *__restrict__ idx,
                                                     uint64_t count, int32_t *__restrict__ x,
                                                     int32_t *__restrict__ y) {
    __shared__ uint8_t sox[256], soy[256], shl[256];
    extern __shared__ __align__(16) uint8_t onehot[];  // 256 items x 32 * ktiles bytes
    load_small_tables(P, sox, soy, shl);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t KB = 32 * M.ktiles;
    // A fragments for every K tile: lane holds A[lane % 16][8 (lane / 16) + 32 kt ..+8]
    long afrag[8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt)
        afrag[kt] = kt < int(M.ktiles)
                        ? *reinterpret_cast<const long *>(M.A + (lane % 16) * KB + 8 * (lane / 16) + 32 * kt)
                        : 0;
    uint8_t *row = onehot + tid * KB;
    const uint64_t ngroups = (count + 255) / 256;
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t t = g * 256 + tid;
        const bool valid = t < count;
        const uint64_t i = valid ? (idx ? uint64_t(idx[t]) : t) : 0;
        const bool inr = valid && i <= P.cells_m1;
        // one-hot digits: byte mu * k + d_mu = 1
        for (uint32_t o = 0; o < KB; o += 16) *reinterpret_cast<uint4 *>(row + o) = make_uint4(0, 0, 0, 0);
        uint32_t ii = inr ? uint32_t(i) : 0;
        for (uint32_t mu = 0; mu < P.r; ++mu) {
            const uint32_t q = udiv(P.divk, ii);
            row[mu * P.k + (ii - q * P.k)] = 1;
            ii = q;
        }
        __syncthreads();
        // the wave's 64 items = 4 groups of 16
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            v4i32 acc = {0, 0, 0, 0};
            const uint8_t *col = onehot + (wave * 64 + grp * 16 + lane % 16) * KB + 8 * (lane / 16);
#pragma unroll
            for (int kt = 0; kt < 8; ++kt)
                if (kt < int(M.ktiles))
                    acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(afrag[kt], *reinterpret_cast<const long *>(col + 32 * kt),
                                                               acc, 0, 0, 0);
            // rows 4 q + r of item lane % 16 in lane (lane % 16) + 16 q
            const uint32_t v = uint32_t(acc[0]) + (uint32_t(acc[1]) << 7) + (uint32_t(acc[2]) << 14) +
                               (uint32_t(acc[3]) << 21);
            const uint64_t item = g * 256 + wave * 64 + grp * 16 + lane % 16;
            if (lane < 32 && item < count) {
                const uint64_t ir = idx ? uint64_t(idx[item]) : item;
                const int32_t out = ir <= P.cells_m1 ? int32_t(v) : -1;
                if (lane < 16) x[item] = out;
                else y[item] = out;
            }
        }
        __syncthreads();
    }
}

// nu with the per-level sum on the matrix cores: each lane takes one item,
// extracts its r digit pairs (as k_nu_digits) and writes the one-hot bytes of
// their replica ids; D = Anu B gives the five 7-bit planes of the index in
// rows 0-4, i.e. rows 0-3 in lanes 0-15 and row 4 in lanes 16-31 of each
// 16-item group, which one cross-lane read brings together.
__global__ __launch_bounds__(256) void k_nu_mfma(MapParams P, MfmaLambda M, const int32_t *__restrict__ x,
                                                 const int32_t *__restrict__ y, uint64_t count,
                                                 uint32_t *__restrict__ idx) {
    __shared__ uint8_t sox[256], soy[256], shl[256];
    __shared__ uint8_t sbad[256];                      // item outside the fractal
    extern __shared__ __align__(16) uint8_t onehot[];  // 256 items x 32 * ktiles bytes
    load_small_tables(P, sox, soy, shl);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t KB = 32 * M.ktiles;
    long afrag[8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt)
        afrag[kt] = kt < int(M.ktiles)
                        ? *reinterpret_cast<const long *>(M.Anu + (lane % 16) * KB + 8 * (lane / 16) + 32 * kt)
                        : 0;
    uint8_t *row = onehot + tid * KB;
    const uint64_t ngroups = (count + 255) / 256;
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t t = g * 256 + tid;
        const int32_t X = t < count ? x[t] : -1, Y = t < count ? y[t] : -1;
        bool bad = uint32_t(X) >= P.n || uint32_t(Y) >= P.n;
        for (uint32_t o = 0; o < KB; o += 16) *reinterpret_cast<uint4 *>(row + o) = make_uint4(0, 0, 0, 0);
        uint32_t ux = bad ? 0u : uint32_t(X), uy = bad ? 0u : uint32_t(Y);
        for (uint32_t mu = 0; mu < P.r; ++mu) {
            const uint32_t qx = udiv(P.divs, ux), qy = udiv(P.divs, uy);
            const uint32_t h = shl[(ux - qx * P.s) + P.s * (uy - qy * P.s)];
            bad |= h == 0xFFu;
            row[mu * P.k + (h == 0xFFu ? 0u : h)] = 1;
            ux = qx;
            uy = qy;
        }
        sbad[tid] = bad;
        __syncthreads();
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            v4i32 acc = {0, 0, 0, 0};
            const uint32_t it = wave * 64 + grp * 16 + lane % 16;  // item within the work-group's 256
            const uint8_t *col = onehot + it * KB + 8 * (lane / 16);
#pragma unroll
            for (int kt = 0; kt < 8; ++kt)
                if (kt < int(M.ktiles))
                    acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(afrag[kt], *reinterpret_cast<const long *>(col + 32 * kt),
                                                               acc, 0, 0, 0);
            // planes 0-3 here (lanes 0-15), plane 4 in lane + 16; the index is
            // below 2^32, so the sum wraps to it exactly
            const uint32_t p4 = uint32_t(__shfl(acc[0], int((lane & 15) + 16)));
            const uint32_t v = uint32_t(acc[0]) + (uint32_t(acc[1]) << 7) + (uint32_t(acc[2]) << 14) +
                               (uint32_t(acc[3]) << 21) + (p4 << 28);
            const uint64_t item = g * 256 + it;
            if (lane < 16 && item < count) idx[item] = sbad[it] ? kOutside : v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Initial state: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) output number
// key = y*n + x of the stream seeded with `seed`; alive iff its top 24 bits
// are below thr = floor(p 2^24) and the cell is a fractal member.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t key) {
    uint64_t z = seed + (key + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t alive_draw(uint64_t seed, uint32_t thr, uint32_t n, uint32_t x,
                                               uint32_t y) {
    uint64_t key = uint64_t(y) * n + x;
    return uint32_t(splitmix64_at(seed, key) >> 40) < thr ? 1u : 0u;
}

__global__ __launch_bounds__(512) void k_init_compact(MapParams P, uint32_t lam_words,
                                                      uint8_t *__restrict__ st, uint64_t seed,
                                                      uint32_t thr) {
    extern __shared__ __align__(16) uint32_t smem_i[];
    load_map_tables(P, lam_words, 0, smem_i, nullptr);
    const uint64_t cells = uint64_t(P.cells_m1) + 1;
    const uint64_t chunks = (cells + 15) / 16;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t c = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < chunks; c += stride) {
        uint32_t w[4] = {0, 0, 0, 0};
        uint64_t base = c * 16;
        for (int b = 0; b < 16; ++b) {
            if (base + b >= cells) break;
            uint32_t x, y;
            lam_lut(P, smem_i, uint32_t(base + b), x, y);
            w[b >> 2] |= alive_draw(seed, thr, P.n, x, y) << (8 * (b & 3));
        }
        if (base + 16 <= cells) {
            *reinterpret_cast<uint4 *>(st + base) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            for (uint64_t b = 0; base + b < cells; ++b) st[base + b] = uint8_t(w[b >> 2] >> (8 * (b & 3)));
        }
    }
}

// Membership of the 16 cells x0..x0+15 of row y as a 16-bit mask (bit j =
// cell x0 + j), from the low-level bitmap and the high-level byte map.
struct BoxLane {
    uint32_t xl, xh, straddle_shift, colmask;
    bool straddle;
};
__device__ __forceinline__ BoxLane box_lane(const BoxParams &B, uint32_t x0) {
    BoxLane L;
    L.xh = udiv(B.divSL, x0);
    L.xl = x0 - L.xh * B.SL;
    L.straddle = (L.xl + 16 > B.SL) && (L.xh + 1 < B.NH);
    L.straddle_shift = B.SL - L.xl;
    uint32_t valid = x0 < B.n ? min(16u, B.n - x0) : 0u;
    L.colmask = valid >= 16 ? 0xFFFFu : ((1u << valid) - 1u);
    return L;
}
__device__ __forceinline__ uint32_t box_member16(const BoxParams &B, const BoxLane &L, uint32_t y) {
    uint32_t yh = udiv(B.divSL, y);
    uint32_t yl = y - yh * B.SL;
    const uint32_t *row = B.low + size_t(yl) * B.LW;
    uint32_t wa = row[L.xl >> 5], wb = row[(L.xl >> 5) + 1];
    uint32_t m = __builtin_amdgcn_alignbit(wb, wa, L.xl & 31) & 0xFFFFu;
    if (L.xh >= B.NH || !B.high[size_t(yh) * B.NH + L.xh]) m = 0;
    if (L.straddle && B.high[size_t(yh) * B.NH + L.xh + 1]) m |= (row[0] << L.straddle_shift) & 0xFFFFu;
    return m & L.colmask;
}

__global__ __launch_bounds__(256) void k_init_box(BoxParams B, uint8_t *__restrict__ st,
                                                  uint64_t seed, uint32_t thr) {
    const uint32_t x0 = (blockIdx.x * 256 + threadIdx.x) * 16;
    if (x0 >= B.pitch) return;
    const BoxLane L = box_lane(B, x0);
    const uint32_t y0 = blockIdx.y * B.rows_per_wg;
    const uint32_t y1 = min(y0 + B.rows_per_wg, B.n);
    for (uint32_t y = y0; y < y1; ++y) {
        uint32_t m = box_member16(B, L, y);
        uint32_t w[4] = {0, 0, 0, 0};
        for (int j = 0; j < 16; ++j)
            if ((m >> j) & 1u) w[j >> 2] |= alive_draw(seed, thr, B.n, x0 + j, y) << (8 * (j & 3));
        *reinterpret_cast<uint4 *>(st + uint64_t(y) * B.pitch + x0) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// ---------------------------------------------------------------------------
// Layout conversion: box <-> compact through lambda.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_zero(uint4 *__restrict__ p, uint64_t n16) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n16; t += stride)
        p[t] = make_uint4(0, 0, 0, 0);
}
__global__ __launch_bounds__(64) void k_fill_tail(uint8_t *__restrict__ p, uint32_t n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(512) void k_expand(MapParams P, uint32_t lam_words,
                                                const uint8_t *__restrict__ compact,
                                                uint8_t *__restrict__ box, uint64_t pitch) {
    extern __shared__ __align__(16) uint32_t smem_e[];
    load_map_tables(P, lam_words, 0, smem_e, nullptr);
    const uint64_t cells = uint64_t(P.cells_m1) + 1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cells; i += stride) {
        uint32_t x, y;
        lam_lut(P, smem_e, uint32_t(i), x, y);
        box[uint64_t(y) * pitch + x] = compact[i];
    }
}

__global__ __launch_bounds__(512) void k_gather(MapParams P, uint32_t lam_words,
                                                const uint8_t *__restrict__ box, uint64_t pitch,
                                                uint8_t *__restrict__ compact) {
    extern __shared__ __align__(16) uint32_t smem_g[];
    load_map_tables(P, lam_words, 0, smem_g, nullptr);
    const uint64_t cells = uint64_t(P.cells_m1) + 1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cells; i += stride) {
        uint32_t x, y;
        lam_lut(P, smem_g, uint32_t(i), x, y);
        compact[i] = box[uint64_t(y) * pitch + x];
    }
}

// ---------------------------------------------------------------------------
// Compact step, one thread per cell: the paper's stencil procedure as
// written (section 3): lambda(i), the eight neighbour coordinates, nu of each,
// read, count, rule.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_step_direct(MapParams P, uint32_t lam_words,
                                                     uint32_t nu_halves,
                                                     const uint8_t *__restrict__ in,
                                                     uint8_t *__restrict__ out, uint32_t rule) {
    extern __shared__ __align__(16) uint32_t smem_d[];
    uint16_t *nu = reinterpret_cast<uint16_t *>(smem_d + lam_words);
    load_map_tables(P, lam_words, nu_halves, smem_d, nu);
    const uint64_t cells = uint64_t(P.cells_m1) + 1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cells; i += stride) {
        uint32_t x, y;
        lam_lut(P, smem_d, uint32_t(i), x, y);
        uint32_t live = 0;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            if (d == 4) continue;
            if ((rule >> 31) && d % 3 != 1 && d / 3 != 1) continue;  // corners: not edge neighbours
            uint32_t j = nu_lut(P, nu, int32_t(x) + d % 3 - 1, int32_t(y) + d / 3 - 1);
            if (j != kOutside) live += in[j];
        }
        uint32_t self = in[i];
        out[i] = uint8_t((rule >> (live + 16 * self)) & 1u);
    }
}

// Rule words with bit 31 set count only the four neighbours that share an
// edge (section 3's example stencil) instead of the eight of the Moore
// neighbourhood; every step kernel honours it.
//
// The lambda approach (section 4, second method): threads run over the
// compact cells but the state lives in the box.  Cell i finds (x, y) =
// lambda(i) and reads its 3 x 3 neighbourhood straight from the box; cells
// outside the fractal hold 0 there, so no nu is needed.  Box cells that are
// not fractal cells are never written.
__global__ __launch_bounds__(512) void k_step_lambda(MapParams P, uint32_t lam_words,
                                                     const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                     uint64_t pitch, uint32_t rule) {
    extern __shared__ __align__(16) uint32_t smem_l[];
    load_map_tables(P, lam_words, 0, smem_l, nullptr);
    const uint64_t cells = uint64_t(P.cells_m1) + 1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cells; i += stride) {
        uint32_t x, y;
        lam_lut(P, smem_l, uint32_t(i), x, y);
        uint32_t sum = 0;
        const bool edge_only = (rule >> 31) != 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const uint32_t yy = y + dy;
            if (yy >= P.n) continue;  // above row 0 wraps to a huge value
            const uint8_t *row = in + uint64_t(yy) * pitch;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (edge_only && dx != 0 && dy != 0) continue;
                const uint32_t xx = x + dx;
                if (xx < P.n) sum += row[xx];
            }
        }
        const uint32_t self = in[uint64_t(y) * pitch + x];
        out[uint64_t(y) * pitch + x] = uint8_t((rule >> (sum - self + 16 * self)) & 1u);
    }
}

// ---------------------------------------------------------------------------
// Blocked layout (section 3, blocked approach: the compact space as a packed
// collection of small bounding boxes): tile t of the tile plan is stored as
// its whole S x S square at bytes [t S^2, (t+1) S^2), cell (x, y) of the
// square at y S + x, positions outside the fractal 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_blocked_scatter(TileParams T, const uint8_t *__restrict__ compact,
                                                         uint8_t *__restrict__ blocked, uint64_t cells) {
    const uint64_t S2 = uint64_t(T.S) * T.S;
    for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < cells; i += uint64_t(gridDim.x) * 256) {
        const uint32_t t = udiv(T.divK, uint32_t(i));
        const uint32_t j = uint32_t(i) - t * T.K;
        blocked[t * S2 + T.blk_pos[j]] = compact[i];
    }
}
__global__ __launch_bounds__(256) void k_blocked_gather(TileParams T, const uint8_t *__restrict__ blocked,
                                                        uint8_t *__restrict__ compact, uint64_t cells) {
    const uint64_t S2 = uint64_t(T.S) * T.S;
    for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < cells; i += uint64_t(gridDim.x) * 256) {
        const uint32_t t = udiv(T.divK, uint32_t(i));
        const uint32_t j = uint32_t(i) - t * T.K;
        compact[i] = blocked[t * S2 + T.blk_pos[j]];
    }
}

// One generation on the blocked layout: a work-group per tile copies the
// tile's square and the facing rows, columns and corners of its eight
// neighbour squares into an LDS box of (S+2) x W bytes, then every thread
// evaluates the rule for four positions at a time (every position of the
// square, the "micro brute force" inside the block) and writes them back,
// member positions only.
template <bool EDGE>
__global__ __launch_bounds__(256) void k_step_blocked(TileParams T, const uint8_t *__restrict__ in,
                                                      uint8_t *__restrict__ out, uint32_t rule, uint32_t W) {
    extern __shared__ __align__(16) uint8_t bbox[];
    const uint32_t S = T.S, nq = (S + 3) >> 2;
    const uint64_t S2 = uint64_t(S) * S;
    const RuleTables RT = rule_tables(rule);
    const uint32_t W4 = W >> 2;
    const uint32_t *box32 = reinterpret_cast<const uint32_t *>(bbox);
    for (uint32_t o = threadIdx.x * 4; o < (S + 2) * W; o += 256 * 4) *reinterpret_cast<uint32_t *>(bbox + o) = 0;
    __syncthreads();
    for (uint64_t t = blockIdx.x; t < T.ntiles; t += gridDim.x) {
        const uint8_t *src = in + t * S2;
        for (uint32_t i = threadIdx.x; i < S * S; i += 256) {
            const uint32_t y = udiv(T.divS, i), x = i - y * S;
            bbox[(y + 1) * W + x + 1] = src[i];
        }
        // the ring: from the neighbour square in direction d (row-major over
        // dy, dx in -1..1 without the centre), 0 where there is none
        for (uint32_t h = threadIdx.x; h < 4 * S + 4; h += 256) {
            int32_t rx, ry;                      // ring position in tile coordinates
            if (h < S) { rx = int32_t(h); ry = -1; }
            else if (h < 2 * S) { rx = int32_t(h - S); ry = int32_t(S); }
            else if (h < 3 * S) { rx = -1; ry = int32_t(h - 2 * S); }
            else if (h < 4 * S) { rx = int32_t(S); ry = int32_t(h - 3 * S); }
            else { const uint32_t c = h - 4 * S; rx = (c & 1) ? int32_t(S) : -1; ry = (c & 2) ? int32_t(S) : -1; }
            const int32_t dx = rx < 0 ? -1 : (rx >= int32_t(S) ? 1 : 0);
            const int32_t dy = ry < 0 ? -1 : (ry >= int32_t(S) ? 1 : 0);
            const uint32_t d = uint32_t((dy + 1) * 3 + (dx + 1));
            const uint32_t nt = T.nbr[t * 8 + (d > 4 ? d - 1 : d)];
            uint8_t v = 0;
            if (nt != kOutside) {
                const uint32_t lx = uint32_t(rx - dx * int32_t(S)), ly = uint32_t(ry - dy * int32_t(S));
                v = in[uint64_t(nt) * S2 + uint64_t(ly) * S + lx];
            }
            bbox[uint32_t(ry + 1) * W + uint32_t(rx + 1)] = v;
        }
        __syncthreads();
        uint8_t *dst = out + t * S2;
        for (uint32_t o = threadIdx.x; o < S * nq; o += 256) {
            const uint32_t y = o / nq, c = o - y * nq;   // row y, columns 4c .. 4c+3
            uint32_t lo[3], hi[3], H[3], C[3];
#pragma unroll
            for (int rr = 0; rr < 3; ++rr) {
                lo[rr] = box32[(y + rr) * W4 + c];
                hi[rr] = box32[(y + rr) * W4 + c + 1];
                C[rr] = alignbyte(hi[rr], lo[rr], 1);
                H[rr] = lo[rr] + C[rr] + alignbyte(hi[rr], lo[rr], 2);
            }
            const uint32_t self = C[1];
            const uint32_t n = EDGE ? C[0] + C[2] + lo[1] + alignbyte(hi[1], lo[1], 2) : H[0] + H[1] + H[2] - self;
            uint32_t next;
            if (RT.perm) {
                const uint32_t born = __builtin_amdgcn_perm(RT.born_hi, RT.born_lo, n);
                const uint32_t surv = __builtin_amdgcn_perm(RT.surv_hi, RT.surv_lo, n);
                const uint32_t smask = __builtin_amdgcn_perm(0u, 0x0000FF00u, self);
                next = (born & ~smask) | (surv & smask);
            } else {
                const uint32_t I = n + (self << 4);
                next = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) next |= __builtin_amdgcn_ubfe(rule, I >> (8 * b), 1) << (8 * b);
            }
            next &= T.blk_mask[o];
            uint8_t *p = dst + y * S + 4 * c;
            const uint32_t nb = min(4u, S - 4 * c);
            if (nb == 4) store_u32(p, next);
            else
                for (uint32_t b = 0; b < nb; ++b) p[b] = uint8_t(next >> (8 * b));
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched step, LDS-resident form for small instances: work-group w owns
// instance w of the launch (steps_of[w] generations, or steps_all for every
// instance if steps_of is NULL; its tile plan from the launch's plan table,
// so instances of every shape share one launch) and runs all of them
// without touching global memory in between.  LDS holds `teams` tile boxes, two copies of the
// instance's state (this generation and the next; tile t at bytes
// [t Kp, t Kp + K), Kp = K rounded up to 16, so every tile starts a 16-byte
// chunk and the phase-0 scatter table serves all of them) and the
// instance's neighbour table.  The work-group splits into `teams` teams of
// 256 / teams threads; per generation the tiles go through in passes of
// `teams` tiles (team j takes tile pass * teams + j), each pass the two
// phases of the tiled step: scatter the tile and its halo from LDS into the
// team's box, then the rule per block with the block's next states written
// in compact order into the other copy.  A thread's scatter offsets, halo
// entries and block corners are the same for every tile and generation, so
// they are loaded once into registers (at most 3 chunks, 5 halo cells and
// 4 blocks per thread; the launcher picks `teams` so they fit).  The final
// state goes to `a` if the instance's generation count is even, else to `b`
// (like the launch-per-generation form, whose ping-pong ends there).
// ---------------------------------------------------------------------------
constexpr uint32_t kResCPT = 3, kResHPT = 5, kResBPT = 4;
template <int BS, bool EDGE>
__device__ __forceinline__ void resident_body(const TileParams &T, const ResidentInstance &I, uint32_t steps,
                                              uint8_t *lds, uint8_t *__restrict__ a, uint8_t *__restrict__ b,
                                              uint32_t rule) {
    const uint32_t tid = threadIdx.x;
    const uint32_t teams = I.teams;
    const uint32_t tsize = 256 / teams;
    const uint32_t team = tid / tsize, lt = tid % tsize;
    const uint32_t K = T.K, Kp = (K + 15) & ~15u, nt = I.ntiles;
    const uint32_t cells = nt * K;
    uint8_t *box = lds + team * T.lds_total;
    uint8_t *cur = lds + teams * T.lds_total;
    uint8_t *nxt = cur + nt * Kp;
    uint32_t *nbrL = reinterpret_cast<uint32_t *>(nxt + nt * Kp);
    const uint64_t base = uint64_t(I.base16) << 4;

    for (uint32_t o = tid * 16; o < teams * T.lds_total; o += 256 * 16)
        *reinterpret_cast<uint4 *>(lds + o) = make_uint4(0, 0, 0, 0);
    for (uint32_t i = tid; i < nt * 8; i += 256) nbrL[i] = I.nbr[i];
    const uint8_t *gin = a + base;
    for (uint32_t i = tid; i < cells; i += 256) {
        const uint32_t t = udiv(T.divK, i);
        cur[t * Kp + (i - t * K)] = gin[i];
    }
    const uint32_t nchunks = Kp >> 4;
    uint4 e[kResCPT][2];
#pragma unroll
    for (uint32_t j = 0; j < kResCPT; ++j) {
        const uint32_t c = min(lt + tsize * j, nchunks - 1);
        e[j][0] = *reinterpret_cast<const uint4 *>(T.lut0p + 16 * c);
        e[j][1] = *reinterpret_cast<const uint4 *>(T.lut0p + 16 * c + 8);
    }
    uint32_t hsrc[kResHPT], hdst[kResHPT], blk[kResBPT];
#pragma unroll
    for (uint32_t j = 0; j < kResHPT; ++j) {
        const uint32_t h = lt + tsize * j;
        const bool ok = h < T.halo_count;
        hsrc[j] = ok ? T.halo_src[h] : kOutside;
        hdst[j] = ok ? T.halo_dst[h] : T.dummy;
    }
#pragma unroll
    for (uint32_t j = 0; j < kResBPT; ++j) blk[j] = T.lut1[min(lt + tsize * j, T.nblk - 1)];
    const RuleTables RT = rule_tables(rule);
    const uint32_t *box32 = reinterpret_cast<const uint32_t *>(box);
    const uint32_t W4 = T.W >> 2;
    __syncthreads();

    for (uint32_t g = 0; g < steps; ++g) {
        for (uint32_t t0 = 0; t0 < nt; t0 += teams) {
            const uint32_t t = t0 + team;
            const bool active = t < nt;
            // 1. the tile and its halo into the team's box (offsets past the
            //    tile's K cells point at the never-read byte)
            if (active) {
                const uint8_t *ct = cur + t * Kp;
#pragma unroll
                for (uint32_t j = 0; j < kResCPT; ++j) {
                    const uint32_t c = lt + tsize * j;
                    if (c < nchunks) {
                        const uint4 v4 = *reinterpret_cast<const uint4 *>(ct + 16 * c);
                        const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
                        const uint32_t ee[8] = {e[j][0].x, e[j][0].y, e[j][0].z, e[j][0].w,
                                                e[j][1].x, e[j][1].y, e[j][1].z, e[j][1].w};
#pragma unroll
                        for (int k = 0; k < 16; ++k)
                            box[(ee[k >> 1] >> (16 * (k & 1))) & 0xFFFFu] = uint8_t(v[k >> 2] >> (8 * (k & 3)));
                    }
                }
#pragma unroll
                for (uint32_t j = 0; j < kResHPT; ++j) {
                    const uint32_t src = hsrc[j];
                    const uint32_t ntile = src != kOutside ? nbrL[t * 8 + (src >> 29)] : kOutside;
                    box[hdst[j]] = ntile != kOutside ? cur[ntile * Kp + (src & 0x1FFFFFFFu)] : uint8_t(0);
                }
            }
            __syncthreads();
            // 2. the rule per block; block bi's CB next states go to cells
            //    [bi CB, (bi + 1) CB) of the tile in the other copy
            if (active) {
                uint8_t *tout = nxt + t * Kp;
#pragma unroll
                for (uint32_t j = 0; j < kResBPT; ++j) {
                    const uint32_t bi = lt + tsize * j;
                    if (bi < T.nblk) {
                        uint32_t next[4];
                        if (RT.perm)
                            block_rows<BS, 1, EDGE>(box32, W4, blk[j], rule, RT, next);
                        else
                            block_rows<BS, 2, EDGE>(box32, W4, blk[j], rule, RT, next);
                        uint32_t w[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            w[d] = __builtin_amdgcn_perm(next[1], next[0], T.pack01[d]);
                            if (BS >= 3) w[d] |= __builtin_amdgcn_perm(next[3], next[2], T.pack23[d]);
                        }
                        uint8_t *p = tout + bi * T.CB;
#pragma unroll
                        for (uint32_t k = 0; k < 16; ++k)
                            if (k < T.CB) p[k] = uint8_t(w[k >> 2] >> (8 * (k & 3)));
                    }
                }
            }
            __syncthreads();
        }
        uint8_t *sw = cur;
        cur = nxt;
        nxt = sw;
    }
    uint8_t *gout = (steps & 1 ? b : a) + base;
    for (uint32_t i = tid; i < cells; i += 256) {
        const uint32_t t = udiv(T.divK, i);
        gout[i] = cur[t * Kp + (i - t * K)];
    }
}
template <bool EDGE>
__global__ __launch_bounds__(256) void k_step_resident(const TileParams *__restrict__ plans,
                                                       const ResidentInstance *__restrict__ inst,
                                                       const uint32_t *__restrict__ steps_of, uint32_t steps_all,
                                                       uint8_t *__restrict__ a, uint8_t *__restrict__ b,
                                                       uint32_t rule) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t steps = steps_of ? steps_of[blockIdx.x] : steps_all;
    if (!steps) return;
    const ResidentInstance I = inst[blockIdx.x];
    const TileParams T = plans[I.plan];
    switch (T.BS) {  // uniform over the work-group
        case 2: resident_body<2, EDGE>(T, I, steps, lds, a, b, rule); break;
        case 3: resident_body<3, EDGE>(T, I, steps, lds, a, b, rule); break;
        default: resident_body<4, EDGE>(T, I, steps, lds, a, b, rule); break;
    }
}

// ---------------------------------------------------------------------------
// Bit-packed compact state: cell i is bit i % 32 of 32-bit word i / 32 (the
// compact order of the byte layout, eight cells per byte, bytes little-endian).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_bits(const uint8_t *__restrict__ bytes, uint32_t *__restrict__ words,
                                                   uint64_t cells, uint64_t nwords) {
    for (uint64_t w = blockIdx.x * 256ull + threadIdx.x; w < nwords; w += uint64_t(gridDim.x) * 256) {
        uint32_t v = 0;
        for (uint32_t b = 0; b < 32; ++b) {
            const uint64_t c = 32 * w + b;
            if (c < cells) v |= uint32_t(bytes[c] != 0) << b;
        }
        words[w] = v;
    }
}
__global__ __launch_bounds__(256) void k_unpack_bits(const uint32_t *__restrict__ words, uint8_t *__restrict__ bytes,
                                                     uint64_t cells, uint64_t nwords) {
    for (uint64_t w = blockIdx.x * 256ull + threadIdx.x; w < nwords; w += uint64_t(gridDim.x) * 256) {
        const uint32_t v = words[w];
        for (uint32_t b = 0; b < 32; ++b) {
            const uint64_t c = 32 * w + b;
            if (c < cells) bytes[c] = uint8_t((v >> b) & 1u);
        }
    }
}

// The tiled step on the packed state.  Per tile (K cells from bit t K, any
// phase within a word): four lanes per word (8 bits each) scatter the tile's
// bits as bytes into the LDS box through a 32-phase copy of lut0 (copy p entry
// j = box offset of local cell j - p, or the never-read byte); the halo bits
// come one per lane; the rule runs per block exactly as in the byte step; a
// block's CB next states, gathered into compact order, become CB bits that
// are OR-ed into an LDS copy of the tile's output words.  Words wholly inside
// the tile are then stored; the first and last words, shared with the
// neighbouring tiles (which other work-groups may be writing), are updated
// with an atomic AND that clears the tile's bits and an atomic OR that sets
// them (the two tiles touch disjoint bits, so the order does not matter).
// Bits past the last cell are never written.  As in the byte step, the
// work-groups are persistent over XCD-contiguous tile ranges and the next
// tile's words, scatter offsets and halo bits are loaded into registers while
// the current one computes; the output-word copy alternates between two LDS
// buffers, so a tile takes two barriers.
constexpr uint32_t kPkWPT = 4, kPkBPT = 4, kPkHPT = 4;  // word quarters, blocks, halo cells per thread
struct PackedPrefetch {
    uint32_t word[kPkWPT];
    uint4 e[kPkWPT];
    uint32_t halo[kPkHPT];
};
// The scatter offsets depend only on the tile's phase (t K mod 32); a
// worker's tiles usually share it (they are a multiple of 32 tiles apart), so
// they are reloaded only when it differs from `pf_ph`, the phase of pf.e.
__device__ __forceinline__ void packed_prefetch(const TileParams &T, const uint16_t *lutw, uint32_t stride,
                                                const uint32_t *in, uint32_t t, const uint32_t (&hsrc)[kPkHPT],
                                                PackedPrefetch &pf, uint32_t &pf_ph) {
    const uint32_t tid = threadIdx.x, K = T.K;
    const uint32_t B = t * K, ph = B & 31, w0 = B >> 5, nq = 4 * ((ph + K + 31) >> 5);
    const uint16_t *lut = lutw + ph * stride;
    const bool reload = ph != pf_ph;  // uniform
    pf_ph = ph;
#pragma unroll
    for (uint32_t j = 0; j < kPkWPT; ++j) {
        const uint32_t l = tid + 256 * j;  // quarter l & 3 of word l >> 2
        if (l < nq) {
            pf.word[j] = in[w0 + (l >> 2)];
            if (reload) pf.e[j] = *reinterpret_cast<const uint4 *>(lut + 8 * l);
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < kPkHPT; ++j) {
        const uint32_t src = hsrc[j];
        const uint32_t ntile = src != kOutside ? T.nbr[uint64_t(t) * 8 + (src >> 29)] : kOutside;
        uint32_t v = 0;
        if (ntile != kOutside) {
            const uint32_t bit = ntile * K + (src & 0x1FFFFFFFu);
            v = (in[bit >> 5] >> (bit & 31)) & 1u;
        }
        pf.halo[j] = v;
    }
}
template <int BS, bool EDGE>
__global__ __launch_bounds__(256) void k_step_packed(TileParams T, const uint16_t *__restrict__ lutw,
                                                     uint32_t lutw_stride, const uint32_t *__restrict__ in,
                                                     uint32_t *__restrict__ out, uint32_t rule) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *box = lds;
    const uint32_t nsw = (T.K + 62) / 32 + 1;  // words of one output copy
    uint32_t *stage0 = reinterpret_cast<uint32_t *>(lds + T.lds_total);
    const uint32_t tid = threadIdx.x, K = T.K;
    for (uint32_t o = tid * 16; o < T.lds_total; o += 256 * 16)
        *reinterpret_cast<uint4 *>(box + o) = make_uint4(0, 0, 0, 0);
    const RuleTables RT = rule_tables(rule);
    uint32_t hsrc[kPkHPT], hdst[kPkHPT], blk[kPkBPT];
#pragma unroll
    for (uint32_t j = 0; j < kPkHPT; ++j) {
        const uint32_t h = tid + 256 * j;
        const bool ok = h < T.halo_count;
        hsrc[j] = ok ? T.halo_src[h] : kOutside;
        hdst[j] = ok ? T.halo_dst[h] : T.dummy;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPkBPT; ++j) blk[j] = T.lut1[min(tid + 256 * j, T.nblk - 1)];
    const uint32_t *box32 = reinterpret_cast<const uint32_t *>(box);
    const uint32_t W4 = T.W >> 2;
    const uint32_t cbmask = T.CB >= 32 ? 0xFFFFFFFFu : (1u << T.CB) - 1;
    const XcdRange R = xcd_range(blockIdx.x, gridDim.x, T.ntiles);
    PackedPrefetch pf;
    uint32_t pf_ph = 0xFFFFFFFFu;  // no offsets loaded yet
    if (R.first < R.end) packed_prefetch(T, lutw, lutw_stride, in, uint32_t(R.first), hsrc, pf, pf_ph);
    __syncthreads();

    uint32_t it = 0;
    for (uint64_t t64 = R.first; t64 < R.end; t64 += R.step, ++it) {
        const uint32_t t = uint32_t(t64);
        const uint32_t B = t * K;  // first cell of the tile (< 2^32)
        const uint32_t ph = B & 31, w0 = B >> 5, nw = (ph + K + 31) >> 5;
        uint32_t *stage = stage0 + (it & 1) * nsw;
        // 1. the tile's bits and its halo into the box; clear the output words
#pragma unroll
        for (uint32_t j = 0; j < kPkWPT; ++j) {
            const uint32_t l = tid + 256 * j;
            if (l < 4 * nw) {
                const uint32_t bits8 = pf.word[j] >> (8 * (l & 3));
                const uint32_t ee[4] = {pf.e[j].x, pf.e[j].y, pf.e[j].z, pf.e[j].w};
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    box[(ee[k >> 1] >> (16 * (k & 1))) & 0xFFFFu] = uint8_t((bits8 >> k) & 1u);
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kPkHPT; ++j) box[hdst[j]] = uint8_t(pf.halo[j]);
        for (uint32_t c = tid; c < nw; c += 256) stage[c] = 0;
        __syncthreads();
        // 2. load the next tile while this one computes
        if (t64 + R.step < R.end)
            packed_prefetch(T, lutw, lutw_stride, in, uint32_t(t64 + R.step), hsrc, pf, pf_ph);
        // 3. the rule per block; its CB bits into the tile's output words
#pragma unroll
        for (uint32_t j = 0; j < kPkBPT; ++j) {
            const uint32_t bi = tid + 256 * j;
            if (bi < T.nblk) {
                uint32_t next[4];
                if (RT.perm)
                    block_rows<BS, 1, EDGE>(box32, W4, blk[j], rule, RT, next);
                else
                    block_rows<BS, 2, EDGE>(box32, W4, blk[j], rule, RT, next);
                uint32_t bits = 0;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    uint32_t w = __builtin_amdgcn_perm(next[1], next[0], T.pack01[d]);
                    if (BS >= 3) w |= __builtin_amdgcn_perm(next[3], next[2], T.pack23[d]);
                    // four 0/1 bytes -> four bits (the partial products never overlap)
                    bits |= ((w * 0x01020408u) >> 24 & 0xFu) << (4 * d);
                }
                bits &= cbmask;
                const uint32_t pos = ph + bi * T.CB, sh = pos & 31;
                atomicOr(&stage[pos >> 5], bits << sh);
                if (sh + T.CB > 32) atomicOr(&stage[(pos >> 5) + 1], bits >> (32 - sh));
            }
        }
        __syncthreads();
        // 4. the output words: whole ones stored, the two shared ones merged
        //    (the box and this copy are next written after the next barrier
        //    and two tiles on, respectively)
        for (uint32_t c = tid; c < nw; c += 256) {
            const uint32_t lo = c == 0 ? ph : 0;
            const uint32_t hi = c + 1 == nw ? ((ph + K - 1) & 31) + 1 : 32;
            const uint32_t mask = (hi == 32 ? 0xFFFFFFFFu : (1u << hi) - 1) & ~((1u << lo) - 1);
            const uint32_t v = stage[c];
            if (mask == 0xFFFFFFFFu) {
                out[w0 + c] = v;
            } else {
                atomicAnd(&out[w0 + c], ~mask);
                atomicOr(&out[w0 + c], v & mask);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Bounding-box step (section 4, method 1): every cell of the n x n box is
// visited.  A thread owns 16 consecutive columns and walks down a band of
// rows, keeping the horizontal 3-sums of three rows in registers, so each
// input byte is fetched once per band.  Non-member cells come out 0.
// ---------------------------------------------------------------------------
struct Row16 {
    uint32_t w[4];
    uint32_t h[4];  // horizontal 3-sums (cols x-1..x+1) per byte
};
__device__ __forceinline__ Row16 load_row16(const BoxParams &B, const uint8_t *__restrict__ in,
                                            uint32_t x0, int64_t y) {
    Row16 r;
    if (y < 0 || y >= int64_t(B.n)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) r.w[i] = r.h[i] = 0;
        return r;
    }
    const uint8_t *row = in + uint64_t(y) * B.pitch;
    const uint4 c = *reinterpret_cast<const uint4 *>(row + x0);
    const uint32_t left = x0 > 0 ? *reinterpret_cast<const uint32_t *>(row + x0 - 4) : 0u;
    const uint32_t right = x0 + 16 < B.pitch ? *reinterpret_cast<const uint32_t *>(row + x0 + 16) : 0u;
    r.w[0] = c.x; r.w[1] = c.y; r.w[2] = c.z; r.w[3] = c.w;
    const uint32_t ext[6] = {left, c.x, c.y, c.z, c.w, right};
#pragma unroll
    for (int i = 0; i < 4; ++i)
        r.h[i] = alignbyte(ext[i + 1], ext[i], 3) + ext[i + 1] + alignbyte(ext[i + 2], ext[i + 1], 1);
    return r;
}

template <bool B3S23>
__global__ __launch_bounds__(256) void k_step_box(BoxParams B, uint32_t gx,
                                                  const uint8_t *__restrict__ in,
                                                  uint8_t *__restrict__ out, uint32_t rule) {
    const uint32_t G = gridDim.x;
    uint32_t lid = blockIdx.x;
    if (G >= 8) {  // XCD-contiguous order of (band, column group)
        uint32_t x = lid & 7, slot = lid >> 3;
        lid = x * (G >> 3) + min(x, G & 7) + slot;
    }
    const uint32_t by = lid / gx, bx = lid - by * gx;
    const uint32_t x0 = (bx * 256 + threadIdx.x) * 16;
    if (x0 >= B.pitch) return;
    const BoxLane L = box_lane(B, x0);
    const uint32_t y0 = by * B.rows_per_wg;
    const uint32_t y1 = min(y0 + B.rows_per_wg, B.n);
    Row16 up = load_row16(B, in, x0, int64_t(y0) - 1);
    Row16 mid = load_row16(B, in, x0, y0);
    for (uint32_t y = y0; y < y1; ++y) {
        const Row16 dn = load_row16(B, in, x0, int64_t(y) + 1);
        const uint32_t m16 = box_member16(B, L, y);
        uint32_t o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t V = up.h[i] + mid.h[i] + dn.h[i];  // 3x3 sums incl. self
            const uint32_t self = mid.w[i];
            uint32_t res;
            if (B3S23) {
                // born with 3, survives with 2 or 3  <=>  (neighbours | self) == 3
                const uint32_t X = ((V - self) | self) ^ 0x03030303u;
                res = (~(X + 0x7F7F7F7Fu) & 0x80808080u) >> 7;
            } else {
                // neighbours + 16 * self; the four edge neighbours are the
                // cells above and below plus the row's 3-sum minus self
                const uint32_t I = ((rule >> 31) ? up.w[i] + dn.w[i] + mid.h[i] : V) + (self << 4) - self;
                res = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) res |= ((rule >> ((I >> (8 * b)) & 0xFFu)) & 1u) << (8 * b);
            }
            o[i] = res & nibble_to_bytes((m16 >> (4 * i)) & 0xFu);
        }
        *reinterpret_cast<uint4 *>(out + uint64_t(y) * B.pitch + x0) = make_uint4(o[0], o[1], o[2], o[3]);
        up = mid;
        mid = dn;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
hipError_t launch_lambda(const MapParams &P, uint32_t lam_words, const uint32_t *idx, uint64_t count,
                         int32_t *x, int32_t *y, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_lambda, dim3(grid), dim3(512), lam_words * 4, st, P, lam_words, idx, count, x, y);
    return hipGetLastError();
}
hipError_t launch_lambda_digits(const MapParams &P, const uint32_t *idx, uint64_t count, int32_t *x, int32_t *y,
                                int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_lambda_digits, dim3(grid), dim3(512), 0, st, P, idx, count, x, y);
    return hipGetLastError();
}
hipError_t launch_nu_digits(const MapParams &P, const int32_t *x, const int32_t *y, uint64_t count, uint32_t *idx,
                            int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_nu_digits, dim3(grid), dim3(512), 0, st, P, x, y, count, idx);
    return hipGetLastError();
}
hipError_t launch_lambda_mfma(const MapParams &P, const MfmaLambda &M, const uint32_t *idx, uint64_t count,
                              int32_t *x, int32_t *y, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_lambda_mfma, dim3(grid), dim3(256), size_t(256) * 32 * M.ktiles, st, P, M, idx, count, x, y);
    return hipGetLastError();
}
hipError_t launch_nu_mfma(const MapParams &P, const MfmaLambda &M, const int32_t *x, const int32_t *y, uint64_t count,
                          uint32_t *idx, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_nu_mfma, dim3(grid), dim3(256), size_t(256) * 32 * M.ktiles, st, P, M, x, y, count, idx);
    return hipGetLastError();
}
hipError_t launch_nu(const MapParams &P, uint32_t nu_halves, const int32_t *x, const int32_t *y,
                     uint64_t count, uint32_t *idx, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_nu, dim3(grid), dim3(512), nu_halves * 2, st, P, nu_halves, x, y, count, idx);
    return hipGetLastError();
}
hipError_t launch_init_compact(const MapParams &P, uint32_t lam_words, uint8_t *st_, uint64_t seed,
                               uint32_t thr, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_init_compact, dim3(grid), dim3(512), lam_words * 4, st, P, lam_words, st_, seed, thr);
    return hipGetLastError();
}
hipError_t launch_init_box(const BoxParams &B, uint8_t *st_, uint64_t seed, uint32_t thr, hipStream_t st) {
    const uint32_t gx = uint32_t((B.pitch / 16 + 255) / 256);
    const uint32_t gy = (B.n + B.rows_per_wg - 1) / B.rows_per_wg;
    hipLaunchKernelGGL(k_init_box, dim3(gx, gy), dim3(256), 0, st, B, st_, seed, thr);
    return hipGetLastError();
}
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t st) {
    const uint64_t n16 = bytes / 16;
    const uint32_t grid = uint32_t(std::min<uint64_t>((n16 + 255) / 256, 65536));
    if (n16) hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, reinterpret_cast<uint4 *>(p), n16);
    return hipGetLastError();
}
hipError_t launch_fill_tail(void *p, uint32_t bytes, hipStream_t st) {
    if (bytes) hipLaunchKernelGGL(k_fill_tail, dim3(1), dim3(64), 0, st, static_cast<uint8_t *>(p), bytes);
    return hipGetLastError();
}
hipError_t launch_expand(const MapParams &P, uint32_t lam_words, const uint8_t *compact, uint8_t *box,
                         uint64_t pitch, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_expand, dim3(grid), dim3(512), lam_words * 4, st, P, lam_words, compact, box, pitch);
    return hipGetLastError();
}
hipError_t launch_gather(const MapParams &P, uint32_t lam_words, const uint8_t *box, uint64_t pitch,
                         uint8_t *compact, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(512), lam_words * 4, st, P, lam_words, box, pitch, compact);
    return hipGetLastError();
}
hipError_t launch_step_direct(const MapParams &P, uint32_t lam_words, uint32_t nu_halves, const uint8_t *in,
                              uint8_t *out, uint32_t rule, int grid, hipStream_t st) {
    const size_t lds = size_t(lam_words) * 4 + size_t(nu_halves) * 2;
    hipLaunchKernelGGL(k_step_direct, dim3(grid), dim3(512), lds, st, P, lam_words, nu_halves, in, out, rule);
    return hipGetLastError();
}
hipError_t launch_blocked_scatter(const TileParams &T, const uint8_t *compact, uint8_t *blocked, uint64_t cells,
                                  int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_blocked_scatter, dim3(grid), dim3(256), 0, st, T, compact, blocked, cells);
    return hipGetLastError();
}
hipError_t launch_blocked_gather(const TileParams &T, const uint8_t *blocked, uint8_t *compact, uint64_t cells,
                                 int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_blocked_gather, dim3(grid), dim3(256), 0, st, T, blocked, compact, cells);
    return hipGetLastError();
}
hipError_t launch_step_blocked(const TileParams &T, const uint8_t *in, uint8_t *out, uint32_t rule, int cu_count,
                               hipStream_t st) {
    const uint32_t W = ((T.S + 2 + 3) & ~3u) + 4;  // dword rows; reads reach column 4 nq + 3
    const size_t lds = size_t(T.S + 2) * W;
    const uint64_t grid = std::min<uint64_t>(T.ntiles, uint64_t(cu_count) * 8);
    if (rule >> 31)
        hipLaunchKernelGGL(k_step_blocked<true>, dim3(uint32_t(grid)), dim3(256), lds, st, T, in, out, rule, W);
    else
        hipLaunchKernelGGL(k_step_blocked<false>, dim3(uint32_t(grid)), dim3(256), lds, st, T, in, out, rule, W);
    return hipGetLastError();
}
hipError_t launch_step_lambda(const MapParams &P, uint32_t lam_words, const uint8_t *in, uint8_t *out,
                              uint64_t pitch, uint32_t rule, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_step_lambda, dim3(grid), dim3(512), size_t(lam_words) * 4, st, P, lam_words, in, out,
                       pitch, rule);
    return hipGetLastError();
}
template <bool BATCH>
static hipError_t launch_tiled_any(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                                   uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    const bool edge = (rule >> 31) != 0;  // four edge neighbours only
    if (T.team == 64)
        return edge ? launch_tiled_inst<BATCH, 64, true>(P, T, in, out, rule, rec, cu_count, st)
                    : launch_tiled_inst<BATCH, 64, false>(P, T, in, out, rule, rec, cu_count, st);
    if (T.team == 256)
        return edge ? launch_tiled_inst<BATCH, 256, true>(P, T, in, out, rule, rec, cu_count, st)
                    : launch_tiled_inst<BATCH, 256, false>(P, T, in, out, rule, rec, cu_count, st);
    return hipErrorInvalidValue;
}
// Most resident work-groups per CU of the edge-record step (0: as many as
// fit), for plans of one block per thread and of more.  Measured with loads
// two tiles ahead: triangle r16 (one block per thread) 20.4 us per
// generation with eight resident or seven; carpet r9 (two) 50.9 with eight,
// 52.1 with seven, 53.2 with six.
#ifndef NBB_EDGES_MAX_PER_CU_ONE
#define NBB_EDGES_MAX_PER_CU_ONE 8
#endif
#ifndef NBB_EDGES_MAX_PER_CU
#define NBB_EDGES_MAX_PER_CU 8
#endif
static constexpr EdgeCaps kEdgesCaps{NBB_EDGES_MAX_PER_CU_ONE, NBB_EDGES_MAX_PER_CU};
hipError_t launch_step_edges(const EdgeParams &E0, uint32_t BS, uint32_t nsrc, const uint8_t *in, uint8_t *out,
                             uint64_t limit, uint32_t rule, const uint32_t *rec, int cu_count, hipStream_t st) {
    EdgeParams E = E0;
    E.limit = limit;
    const bool edge = (rule >> 31) != 0;
    const int kind = edges_rule_kind(rule);
    const EdgeCaps mx = kEdgesCaps;
#define NBB_EDGES_GO(B)                                                                                  \
    do {                                                                                                  \
        if (edge) return launch_edges_inst<B, true, 1>(E, BS, nsrc, in, out, rule, rec, cu_count, mx, st); \
        if (kind == 0) return launch_edges_inst<B, false, 0>(E, BS, nsrc, in, out, rule, rec, cu_count, mx, st); \
        if (kind == 1) return launch_edges_inst<B, false, 1>(E, BS, nsrc, in, out, rule, rec, cu_count, mx, st); \
        return launch_edges_inst<B, false, 2>(E, BS, nsrc, in, out, rule, rec, cu_count, mx, st);          \
    } while (0)
    if (rec) NBB_EDGES_GO(true);
    NBB_EDGES_GO(false);
#undef NBB_EDGES_GO
}
hipError_t launch_step_tiled(const MapParams &P, const TileParams &T, const uint8_t *in, uint8_t *out,
                             uint32_t rule, int cu_count, hipStream_t st) {
    return launch_tiled_any<false>(P, T, in, out, rule, nullptr, cu_count, st);
}
hipError_t launch_step_tiled_batch(const TileParams &T, const uint32_t *rec, const uint8_t *arena_in,
                                   uint8_t *arena_out, uint32_t rule, int cu_count, hipStream_t st) {
    return launch_tiled_any<true>(MapParams{}, T, arena_in, arena_out, rule, rec, cu_count, st);
}
uint32_t resident_lds_bytes(const TileParams &T, uint32_t ntiles, uint32_t teams) {
    const uint64_t Kp = (T.K + 15) & ~15u;
    const uint64_t n = uint64_t(teams) * T.lds_total + 2 * ntiles * Kp + 32 * uint64_t(ntiles);
    return n > 0xFFFFFFFFu ? 0xFFFFFFFFu : uint32_t(n);
}
bool resident_fits(const TileParams &T, uint32_t teams) {
    const uint32_t tsize = 256 / teams;
    const uint32_t nchunks = (T.K + 15) >> 4;
    return teams && 256 % teams == 0 && nchunks <= kResCPT * tsize && T.halo_count <= kResHPT * tsize &&
           T.nblk <= kResBPT * tsize;
}
hipError_t launch_step_resident(const TileParams *plans, const ResidentInstance *inst, uint32_t count,
                                const uint32_t *steps_of, uint32_t steps_all, uint32_t lds, uint8_t *a, uint8_t *b,
                                uint32_t rule, hipStream_t st) {
    if (!count) return hipSuccess;
    if ((rule >> 31) != 0)
        hipLaunchKernelGGL(k_step_resident<true>, dim3(count), dim3(256), lds, st, plans, inst, steps_of, steps_all,
                           a, b, rule);
    else
        hipLaunchKernelGGL(k_step_resident<false>, dim3(count), dim3(256), lds, st, plans, inst, steps_of,
                           steps_all, a, b, rule);
    return hipGetLastError();
}
__global__ __launch_bounds__(256) void k_set_words(uint32_t *__restrict__ dst, WordChunk w, uint32_t n) {
    if (threadIdx.x < n) dst[threadIdx.x] = w.v[threadIdx.x];
}
hipError_t launch_set_words(uint32_t *dst, const uint32_t *src, uint32_t n, hipStream_t st) {
    for (uint32_t i = 0; i < n; i += kWordChunk) {
        WordChunk w{};
        const uint32_t m = std::min(kWordChunk, n - i);
        for (uint32_t j = 0; j < m; ++j) w.v[j] = src[i + j];
        hipLaunchKernelGGL(k_set_words, dim3(1), dim3(kWordChunk), 0, st, dst + i, w, m);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
// One thread per batch tile: find the instance holding batch tile g (the
// last one whose first tile is <= g) and write the tile's record and its
// eight neighbours, copied from the instance's own neighbour table.
__global__ __launch_bounds__(256) void k_batch_tiles(const BatchInstance *__restrict__ inst, uint32_t ninst,
                                                     uint32_t total, uint32_t *__restrict__ rec,
                                                     uint32_t *__restrict__ nbr) {
    for (uint32_t g = blockIdx.x * 256 + threadIdx.x; g < total; g += gridDim.x * 256) {
        uint32_t lo = 0, hi = ninst - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (inst[mid].tile0 <= g) lo = mid;
            else hi = mid - 1;
        }
        const BatchInstance &I = inst[lo];
        const uint32_t t = g - I.tile0;
        rec[2 * uint64_t(g)] = I.base16;
        rec[2 * uint64_t(g) + 1] = t | ((I.tail_partial && t + 1 == I.ntiles) ? 0x80000000u : 0u);
        const uint4 *s4 = reinterpret_cast<const uint4 *>(I.nbr + 8 * uint64_t(t));
        uint4 *d4 = reinterpret_cast<uint4 *>(nbr + 8 * uint64_t(g));
        d4[0] = s4[0];
        d4[1] = s4[1];
    }
}
hipError_t launch_batch_tiles(const BatchInstance *inst, uint32_t ninst, uint32_t total, uint32_t *rec,
                              uint32_t *nbr, hipStream_t st) {
    if (!total || !ninst) return hipSuccess;
    const uint32_t grid = std::min<uint32_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_batch_tiles, dim3(grid), dim3(256), 0, st, inst, ninst, total, rec, nbr);
    return hipGetLastError();
}
hipError_t launch_pack_bits(const uint8_t *bytes, uint32_t *words, uint64_t cells, int grid, hipStream_t st) {
    const uint64_t nwords = (cells + 31) / 32;
    if (!nwords) return hipSuccess;
    hipLaunchKernelGGL(k_pack_bits, dim3(grid), dim3(256), 0, st, bytes, words, cells, nwords);
    return hipGetLastError();
}
hipError_t launch_unpack_bits(const uint32_t *words, uint8_t *bytes, uint64_t cells, int grid, hipStream_t st) {
    const uint64_t nwords = (cells + 31) / 32;
    if (!nwords) return hipSuccess;
    hipLaunchKernelGGL(k_unpack_bits, dim3(grid), dim3(256), 0, st, words, bytes, cells, nwords);
    return hipGetLastError();
}
uint32_t packed_stage_words(const TileParams &T) { return 2 * ((T.K + 62) / 32 + 1); }
bool packed_fits(const TileParams &T) {
    return T.nblk <= kPkBPT * 256 && T.halo_count <= kPkHPT * 256 && T.CB <= 16 &&
           4 * ((T.K + 62) / 32) <= kPkWPT * 256 && T.lds_total + 4 * packed_stage_words(T) <= 65536;
}
// Persistent launch: as many work-groups as can be resident at once.
template <int BS, bool EDGE>
static hipError_t launch_packed_t(const TileParams &T, const uint16_t *lutw, uint32_t stride, const uint32_t *in,
                                  uint32_t *out, uint32_t rule, int cu_count, hipStream_t st) {
    const uint32_t lds = T.lds_total + 4 * packed_stage_words(T);
    static std::atomic<uint64_t> cached{0};  // lds << 32 | per_cu
    int per_cu = 0;
    const uint64_t c = cached.load(std::memory_order_relaxed);
    if (c >> 32 == lds && (c & 0xFFFFFFFFu)) {
        per_cu = int(c & 0xFFFFFFFFu);
    } else {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_packed<BS, EDGE>, 256, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        cached.store(uint64_t(lds) << 32 | uint32_t(per_cu), std::memory_order_relaxed);
    }
    const uint32_t grid = uint32_t(std::min<uint64_t>(T.ntiles, uint64_t(per_cu) * cu_count));
    hipLaunchKernelGGL((k_step_packed<BS, EDGE>), dim3(grid), dim3(256), lds, st, T, lutw, stride, in, out, rule);
    return hipGetLastError();
}
hipError_t launch_step_packed(const TileParams &T, const uint16_t *lutw, uint32_t stride, const uint32_t *in,
                              uint32_t *out, uint32_t rule, int cu_count, hipStream_t st) {
    if (!packed_fits(T) || stride % 32 || stride < 32 * ((T.K + 62) / 32)) return hipErrorInvalidValue;
    if (!T.ntiles) return hipSuccess;
    const bool edge = (rule >> 31) != 0;
    switch (T.BS) {
        case 2: return edge ? launch_packed_t<2, true>(T, lutw, stride, in, out, rule, cu_count, st)
                            : launch_packed_t<2, false>(T, lutw, stride, in, out, rule, cu_count, st);
        case 3: return edge ? launch_packed_t<3, true>(T, lutw, stride, in, out, rule, cu_count, st)
                            : launch_packed_t<3, false>(T, lutw, stride, in, out, rule, cu_count, st);
        case 4: return edge ? launch_packed_t<4, true>(T, lutw, stride, in, out, rule, cu_count, st)
                            : launch_packed_t<4, false>(T, lutw, stride, in, out, rule, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_step_box(const BoxParams &B, const uint8_t *in, uint8_t *out, uint32_t rule, hipStream_t st) {
    const uint32_t gx = uint32_t((B.pitch / 16 + 255) / 256);
    const uint32_t gy = (B.n + B.rows_per_wg - 1) / B.rows_per_wg;
    const uint32_t G = gx * gy;
    if (rule == ((1u << 3) | ((1u << 2 | 1u << 3) << 16)))
        hipLaunchKernelGGL(k_step_box<true>, dim3(G), dim3(256), 0, st, B, gx, in, out, rule);
    else
        hipLaunchKernelGGL(k_step_box<false>, dim3(G), dim3(256), 0, st, B, gx, in, out, rule);
    return hipGetLastError();
}

}  // namespace nbb
