/* The C oracle over 300 random NBB fractals (s 2..4, any k, r <= 5, both
 * neighbourhoods) under AddressSanitizer and UndefinedBehaviorSanitizer, run
 * by tests/test_sanitizers.py: init, compact step, box step, gather/expand,
 * light-cone cells and nu(lambda(i)) = i; the compact step must equal the
 * gathered box step. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
size_t orc_fractal_size(void);
int orc_make(void *f, int64_t k, int64_t s, const int32_t *offsets, int64_t r);
void orc_lambda(const void *f, int64_t i, int64_t *x, int64_t *y);
int64_t orc_nu(const void *f, int64_t x, int64_t y);
void orc_init_compact(const void *f, uint8_t *state, uint64_t seed, double p);
void orc_init_bbox(const void *f, uint8_t *state, uint64_t seed, double p);
void orc_member_mask(const void *f, uint8_t *mask);
void orc_bbox_step(const void *f, const uint8_t *mask, const uint8_t *in, uint8_t *out, uint32_t rule);
void orc_compact_step(const void *f, const uint8_t *in, uint8_t *out, uint32_t rule);
void orc_cells_after(const void *f, const uint8_t *in, const int64_t *idx, int64_t count, uint32_t rule, int steps,
                     uint8_t *out);
void orc_gather(const void *f, const uint8_t *bbox, uint8_t *compact);
void orc_expand(const void *f, const uint8_t *compact, uint8_t *bbox);
int main(void) {
    srand(7);
    void *f = malloc(orc_fractal_size());
    int checked = 0;
    for (int it = 0; it < 300; ++it) {
        int s = 2 + rand() % 3, k = 1 + rand() % (s * s), r = rand() % 6;
        int cells[16], off[32];
        for (int i = 0; i < s * s; ++i) cells[i] = i;
        for (int i = s * s - 1; i > 0; --i) { int j = rand() % (i + 1); int t = cells[i]; cells[i] = cells[j]; cells[j] = t; }
        for (int j = 0; j < k; ++j) { off[2 * j] = cells[j] % s; off[2 * j + 1] = cells[j] / s; }
        if (orc_make(f, k, s, off, r)) continue;
        int64_t n = 1, c = 1;
        for (int i = 0; i < r; ++i) { n *= s; c *= k; }
        if (n * n > 300000) continue;
        uint8_t *a = malloc(c), *b = malloc(c), *box = malloc(n * n), *box2 = malloc(n * n), *mask = malloc(n * n);
        uint32_t rule = (1u << 3) | ((1u << 2 | 1u << 3) << 16);
        if (it & 1) rule |= 1u << 31;
        orc_init_compact(f, a, it, 0.5);
        orc_compact_step(f, a, b, rule);
        orc_expand(f, a, box);
        orc_member_mask(f, mask);
        orc_bbox_step(f, mask, box, box2, rule);
        uint8_t *g = malloc(c);
        orc_gather(f, box2, g);
        if (memcmp(g, b, c)) { printf("mismatch it=%d\n", it); return 1; }
        int64_t idx[4] = {0, c - 1, c / 2, c / 3};
        uint8_t o4[4];
        orc_cells_after(f, a, idx, 4, rule, 2, o4);
        for (int64_t i = 0; i < c; i += 1 + c / 50) {
            int64_t x, y; orc_lambda(f, i, &x, &y);
            if (orc_nu(f, x, y) != i) { printf("nu(lambda) it=%d\n", it); return 1; }
        }
        (void)orc_nu(f, -1, 0); (void)orc_nu(f, n, n);
        orc_init_bbox(f, box, it, 0.3);
        free(a); free(b); free(box); free(box2); free(mask); free(g);
        ++checked;
    }
    printf("checked %d\n", checked);
    free(f);
    return 0;
}
