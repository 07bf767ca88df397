/*
 * Runs every function of the CPU oracle (oracle/sco.c) on small seeded images of many shapes
 * under AddressSanitizer and UndefinedBehaviorSanitizer, with every buffer sized exactly as the
 * oracle's comments state, plus its argument errors.  Exit status 0 = every call returned what
 * was expected; the sanitizers abort on a finding.  Test infrastructure only: built by
 * tests/test_sanitize.py.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int sco_energy(const uint8_t*, int, int, int, int, int32_t*);
int sco_dp(const int32_t*, int, int, int64_t*, uint8_t*, int32_t*, int64_t*);
int sco_remove_seam(uint8_t*, int, int, int, int, const int32_t*);
int sco_carve(uint8_t*, int, int, int, int, int, int32_t*, int64_t*);
int sco_seam_origins(const int32_t*, int, int, int, int32_t*);
int sco_insert_seams(const uint8_t*, int, int, int, int, int, uint8_t*, int, int32_t*);
int sco_forward_dp(const uint8_t*, int, int, int, int, int64_t*, uint8_t*, int32_t*, int64_t*);
int sco_carve_forward(uint8_t*, int, int, int, int, int, int32_t*, int64_t*);
int sco_transpose(const uint8_t*, int, int, int, int, uint8_t*, int);
int sco_carve_hv(uint8_t*, int, int, int, int, int, int, uint8_t*, int, int32_t*, int64_t*, int32_t*, int64_t*);
int sco_greedy_seam(const int32_t*, int, int, int32_t*, int64_t*);
int sco_brute_seam(const int32_t*, int, int, int32_t*, int64_t*);
int32_t sco_mask_bias(int, int);
int sco_object_direction(const uint8_t*, int, int, int);
int sco_masked_seam(const uint8_t*, const uint8_t*, int, int, int, int, int, int32_t, int32_t*, int64_t*);
int sco_remove_object(const uint8_t*, const uint8_t*, int, int, int, int, int, int, int, uint8_t*, int, int32_t*,
                      int32_t*, int64_t*);

static int g_fail = 0;
#define EXPECT(c)                                                                        \
    do {                                                                                 \
        if (!(c)) {                                                                      \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                                    \
        }                                                                                \
    } while (0)

static uint64_t g_x = 0x9E3779B97F4A7C15ull;
static int rnd(int lo, int hi) {
    g_x ^= g_x << 13;
    g_x ^= g_x >> 7;
    g_x ^= g_x << 17;
    return lo + (int)(g_x % (uint64_t)(hi - lo + 1));
}

/* exactly-sized heap buffers, so any overrun is a sanitizer finding */
static void* xmalloc(size_t n) {
    void* p = malloc(n ? n : 1);
    if (!p) abort();
    return p;
}

static void one_shape(int H, int W, int C, int pad, int alpha) {
    const int pitch = W * C + pad, n = H * pitch;
    uint8_t* img = xmalloc((size_t)n);
    for (int i = 0; i < n; ++i) img[i] = (uint8_t)rnd(0, alpha - 1);
    int32_t* e = xmalloc(sizeof(int32_t) * (size_t)H * W);
    EXPECT(sco_energy(img, H, W, C, pitch, e) == 0);
    int64_t* M = xmalloc(sizeof(int64_t) * (size_t)H * W);
    uint8_t* D = xmalloc((size_t)H * W);
    int32_t* seam = xmalloc(sizeof(int32_t) * (size_t)H);
    int64_t cost = 0, gcost = 0;
    EXPECT(sco_dp(e, H, W, M, D, seam, &cost) == 0);
    EXPECT(sco_dp(e, H, W, NULL, NULL, seam, &cost) == 0);
    EXPECT(sco_greedy_seam(e, H, W, seam, &gcost) == 0 && cost <= gcost);
    if (H <= 7 && W <= 7) {
        int64_t bcost = 0;
        EXPECT(sco_brute_seam(e, H, W, seam, &bcost) == 0 && bcost == cost);
    }
    EXPECT(sco_forward_dp(img, H, W, C, pitch, M, D, seam, &cost) == 0);
    const int tw = rnd(1, W), k = W - tw;
    int32_t* seams = xmalloc(sizeof(int32_t) * (size_t)(k ? k : 1) * H);
    int64_t* costs = xmalloc(sizeof(int64_t) * (size_t)(k ? k : 1));
    uint8_t* work = xmalloc((size_t)n);
    memcpy(work, img, (size_t)n);
    EXPECT(sco_carve(work, H, W, C, pitch, tw, seams, costs) == 0);
    int32_t* orig = xmalloc(sizeof(int32_t) * (size_t)(k ? k : 1) * H);
    EXPECT(sco_seam_origins(seams, k, H, W, orig) == 0);
    memcpy(work, img, (size_t)n);
    EXPECT(sco_carve_forward(work, H, W, C, pitch, tw, seams, costs) == 0);
    if (k < W) {
        const int ki = rnd(0, W - 1), op = (W + ki) * C;
        uint8_t* out = xmalloc((size_t)H * op);
        int32_t* io = xmalloc(sizeof(int32_t) * (size_t)(ki ? ki : 1) * H);
        EXPECT(sco_insert_seams(img, H, W, C, pitch, ki, out, op, io) == 0);
        free(out);
        free(io);
    }
    uint8_t* tr = xmalloc((size_t)W * H * C);
    EXPECT(sco_transpose(img, H, W, C, pitch, tr, H * C) == 0);
    {
        const int th = rnd(1, H), op = tw * C;
        int32_t* hs = xmalloc(sizeof(int32_t) * (size_t)(H - th ? H - th : 1) * tw);
        int64_t* hc = xmalloc(sizeof(int64_t) * (size_t)(H - th ? H - th : 1));
        uint8_t* out = xmalloc((size_t)th * op);
        memcpy(work, img, (size_t)n);
        EXPECT(sco_carve_hv(work, H, W, C, pitch, tw, th, out, op, seams, costs, hs, hc) == 0);
        free(hs);
        free(hc);
        free(out);
    }
    /* object removal: a random box mask with stray pixels, every direction, with and without restore */
    {
        const int mp = W + rnd(0, 5);
        uint8_t* mask = xmalloc((size_t)H * mp);
        memset(mask, 0, (size_t)H * mp);
        const int y0 = rnd(0, H - 1), x0 = rnd(0, W - 1), y1 = rnd(y0, H - 1), x1 = rnd(x0, W - 1);
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) mask[(size_t)y * mp + x] = (uint8_t)rnd(1, 255);
        for (int s = 0; s < 3; ++s) mask[(size_t)rnd(0, H - 1) * mp + rnd(0, W - 1)] = 1;
        EXPECT(sco_object_direction(mask, H, W, mp) >= 0);
        EXPECT(sco_masked_seam(img, mask, H, W, C, pitch, mp, sco_mask_bias(H, C), seam, &cost) == 0);
        const int op = W * C + rnd(0, 3), mx = H > W ? H : W;
        uint8_t* out = xmalloc((size_t)H * op);
        int32_t info[5];
        int32_t* os = xmalloc(sizeof(int32_t) * (size_t)H * W);
        int64_t* oc = xmalloc(sizeof(int64_t) * (size_t)mx);
        for (int dir = -1; dir <= 1; ++dir)
            for (int restore = 0; restore <= 1; ++restore) {
                const int rc = sco_remove_object(img, mask, H, W, C, pitch, mp, dir, restore, out, op, info, os, oc);
                EXPECT(rc == 0 || (restore && rc == -1));  /* a one-column result cannot be restored */
            }
        free(mask);
        free(out);
        free(os);
        free(oc);
    }
    free(img);
    free(e);
    free(M);
    free(D);
    free(seam);
    free(seams);
    free(costs);
    free(orig);
    free(work);
    free(tr);
}

int main(void) {
    for (int t = 0; t < 160; ++t) {
        const int H = rnd(1, 24), W = rnd(1, 24), C = rnd(1, 4);
        one_shape(H, W, C, rnd(0, 7), (t & 1) ? 256 : rnd(2, 4));
    }
    one_shape(48, 64, 3, 0, 256);
    one_shape(1, 1, 1, 0, 256);
    /* argument errors */
    int32_t s[4];
    int64_t c;
    uint8_t b[64] = {0};
    EXPECT(sco_energy(b, 0, 4, 3, 12, s) != 0);
    EXPECT(sco_dp(NULL, 2, 2, NULL, NULL, s, &c) != 0);
    EXPECT(sco_carve(b, 2, 4, 3, 12, 5, NULL, NULL) != 0);
    EXPECT(sco_insert_seams(b, 2, 4, 3, 12, 4, b, 24, NULL) != 0);
    EXPECT(sco_remove_object(b, b, 2, 4, 3, 12, 4, 2, 0, b, 12, s, NULL, NULL) != 0);
    if (g_fail) fprintf(stderr, "%d expectation(s) failed\n", g_fail);
    else printf("oracle driver: all expectations held\n");
    return g_fail ? 1 : 0;
}
