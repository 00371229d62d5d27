// Several generations of the compact step per launch (temporal blocking), for
// instances too small to fill the GPU, where one launch per generation costs
// more than the generation itself.
//
// Section 3's stencil procedure on its blocked approach, taken over several
// generations: tile t (compact cells [t K, (t+1) K), one level-m copy of the
// fractal, an S x S square of the embedding) and every cell of its eight
// neighbour tiles within distance h of the square are scattered into a box of
// side B = S + 2h in LDS, with a member mask (1 where a fractal cell sits);
// the work-group then applies the rule to the whole box `gens` <= h times,
// reading and writing LDS only, and stores the tile's own cells.  A generation
// computed in the box is exact at every position whose 3 x 3 neighbourhood
// was exact before, so the errors that the missing outer ring brings in
// advance by one ring per generation and never reach the square while
// gens <= h.  The rows (and dword columns) within g of the border are not
// computed at generation g: nothing exact depends on them.
//
// Four positions per dword (SWAR; sums never exceed 9, so bytes do not carry):
// a thread owns one dword column of a band of rows and marches down it,
// keeping the horizontal 3-sums of the rows above and at the current row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace nbb {

// RULE: 0 = B3/S23 (born with 3, survives with 2 or 3 <=> (n | self) == 3),
// 1 = rules without birth or survival at 8 (two v_perm table look-ups),
// 2 = any rule (the rule word's bit n + 16 self, per byte).
template <int RULE>
__device__ __forceinline__ uint32_t rule4(uint32_t n, uint32_t self, uint32_t rule, const RuleTables &RT) {
    if (RULE == 0) return __builtin_amdgcn_perm(0u, 0x01000000u, n | self);
    if (RULE == 1) {
        const uint32_t born = __builtin_amdgcn_perm(RT.born_hi, RT.born_lo, n);
        const uint32_t surv = __builtin_amdgcn_perm(RT.surv_hi, RT.surv_lo, n);
        const uint32_t smask = __builtin_amdgcn_perm(0u, 0x0000FF00u, self);  // 0xFF where alive
        return (surv & smask) | (born & ~smask);
    }
    const uint32_t I = n + (self << 4);
    uint32_t v = __builtin_amdgcn_ubfe(rule, I, 1);
#pragma unroll
    for (int c = 1; c < 4; ++c) v |= __builtin_amdgcn_ubfe(rule, I >> (8 * c), 1) << (8 * c);
    return v;
}

template <int RULE, bool EDGE>
__global__ __launch_bounds__(256) void k_step_temporal(TemporalParams T, const uint8_t *__restrict__ in,
                                                       uint8_t *__restrict__ out, uint32_t rule, uint32_t gens) {
    extern __shared__ __align__(16) uint8_t lds_t[];
    const uint32_t tid = threadIdx.x;
    const uint32_t t = blockIdx.x;
    uint8_t *cur = lds_t;
    uint8_t *nxt = lds_t + T.box_bytes;
    const uint32_t *mask32 = reinterpret_cast<const uint32_t *>(lds_t + 2 * T.box_bytes);
    for (uint32_t o = tid * 16; o < 3 * T.box_bytes; o += 256 * 16)
        *reinterpret_cast<uint4 *>(lds_t + o) = make_uint4(0, 0, 0, 0);
    __syncthreads();
    // the tile's cells and the neighbour cells inside the box
    uint8_t *mask = lds_t + 2 * T.box_bytes;
    const uint8_t *src = in + uint64_t(t) * T.K;
    for (uint32_t j = tid; j < T.K; j += 256) {
        const uint32_t o = T.self[j];
        cur[o] = src[j];
        mask[o] = 1;
    }
    const uint32_t *nb = T.nbr + uint64_t(t) * 8;
    for (uint32_t e = tid; e < T.nhalo; e += 256) {
        const uint32_t w = T.halo[2 * e], o = T.halo[2 * e + 1];
        const uint32_t nt = nb[w >> 29];
        if (nt != kOutside) {
            cur[o] = in[uint64_t(nt) * T.K + (w & 0x1FFFFFFFu)];
            mask[o] = 1;
        }
    }
    __syncthreads();
    const RuleTables RT = rule_tables(rule);
    const uint32_t C = T.P >> 2;  // dwords per box row
    for (uint32_t g = 0; g < gens; ++g) {
        // rows [y0, y1) and the dword columns [c0, c1) that cover the same
        // columns; everything nearer the border is left as it is
        const uint32_t y0 = g + 1, y1 = T.B - 1 - g;
        const uint32_t c0 = y0 >> 2, c1 = (y1 + 3) >> 2;
        const uint32_t nc = c1 - c0, nrows = y1 - y0;
        const uint32_t bands = 256 / nc;  // nc <= C <= 64
        const uint32_t c = c0 + tid % nc, band = tid / nc;
        const uint32_t per = (nrows + bands - 1) / bands;
        const uint32_t ya = y0 + band * per, yb = min(y1, ya + per);
        const uint32_t *cur32 = reinterpret_cast<const uint32_t *>(cur);
        uint32_t *nxt32 = reinterpret_cast<uint32_t *>(nxt);
        if (band < bands && ya < yb) {
            // centre dword and left + right neighbours (per byte) of row y
            auto row = [&](uint32_t y, uint32_t &mid, uint32_t &lr) {
                const uint32_t base = y * C + c;
                mid = cur32[base];
                const uint32_t l = c ? cur32[base - 1] : 0u;
                const uint32_t r = c + 1 < C ? cur32[base + 1] : 0u;
                lr = alignbyte(mid, l, 3) + alignbyte(r, mid, 1);
            };
            uint32_t mA, lA, mB, lB;
            row(ya - 1, mA, lA);
            row(ya, mB, lB);
            for (uint32_t y = ya; y < yb; ++y) {
                uint32_t mC, lC;
                row(y + 1, mC, lC);
                const uint32_t n = EDGE ? mA + mC + lB : (mA + lA) + lB + (mC + lC);
                nxt32[y * C + c] = rule4<RULE>(n, mB, rule, RT) & mask32[y * C + c];
                mA = mB;
                lA = lB;
                mB = mC;
                lB = lC;
            }
        }
        __syncthreads();
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    uint8_t *dst = out + uint64_t(t) * T.K;
    for (uint32_t j = tid; j < T.K; j += 256) dst[j] = cur[T.self[j]];
}

template <int RULE, bool EDGE>
static hipError_t launch_temporal_t(const TemporalParams &T, const uint8_t *in, uint8_t *out, uint32_t rule,
                                    uint32_t gens, hipStream_t st) {
    hipLaunchKernelGGL((k_step_temporal<RULE, EDGE>), dim3(T.ntiles), dim3(256), 3 * T.box_bytes, st, T, in, out,
                       rule, gens);
    return hipGetLastError();
}

hipError_t launch_step_temporal(const TemporalParams &T, const uint8_t *in, uint8_t *out, uint32_t rule,
                                uint32_t gens, hipStream_t st) {
    if (!T.ntiles || !gens) return hipSuccess;
    if (T.B < 3 || T.P / 4 > 64 || 2 * T.h + 1 > T.B || gens > T.h) return hipErrorInvalidValue;
    if (rule >> 31) return launch_temporal_t<1, true>(T, in, out, rule, gens, st);
    if (rule == ((1u << 3) | ((1u << 2 | 1u << 3) << 16))) return launch_temporal_t<0, false>(T, in, out, rule, gens, st);
    if ((rule & ((1u << 8) | (1u << 24))) == 0) return launch_temporal_t<1, false>(T, in, out, rule, gens, st);
    return launch_temporal_t<2, false>(T, in, out, rule, gens, st);
}

}  // namespace nbb
