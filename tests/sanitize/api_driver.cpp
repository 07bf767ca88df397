// Exercises the host code of the C ABI (validation, workspace layouts, the batch planner) under
// AddressSanitizer and UndefinedBehaviorSanitizer, with the kernel launchers replaced by the
// stand-ins of kernel_stubs.cpp.  Device pointers are host addresses that the host code never
// dereferences.  Exit status 0 = every expectation held; the sanitizers abort on a finding.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sc.h"

static int g_fail = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)

int main() {
    alignas(256) static uint8_t fake[1 << 16];  // stands for device memory; never dereferenced
    uint8_t* p = fake;
    void* ws = fake;
    const size_t big = (size_t)1 << 40;

    // workspace sizes: zero on bad shapes, monotone in the image size
    EXPECT(sc_workspace_bytes(0, 5, 3) == 0 && sc_workspace_bytes(5, 5, 5) == 0);
    EXPECT(sc_workspace_bytes(1080, 1920, 3) < sc_workspace_bytes(2160, 3840, 3));
    EXPECT(sc_forward_workspace_bytes(7, 9, 1) > 0 && sc_object_workspace_bytes(7, 9, 4, 1) > 0);
    EXPECT(sc_insert_workspace_bytes(10, 10, 3, 30, 10) == 0 && sc_insert_workspace_bytes(10, 10, 3, 30, 9) > 0);
    EXPECT(sc_object_workspace_bytes(0, 9, 3, 0) == 0 && sc_slot_table_bytes(4) > 0);
    for (int v = 0; v <= sc_variant_count(); ++v) EXPECT(sc_variant_name(v) != nullptr);

    // argument errors of every entry point
    EXPECT(sc_energy(p, 0, 5, 3, 15, (int32_t*)p, nullptr) == SC_EINVAL);
    EXPECT(sc_energy(p, 5483, 5, 3, 15, (int32_t*)p, nullptr) == SC_EUNSUPPORTED);
    EXPECT(sc_dp_seam((int32_t*)p, 4, 4, (int32_t*)p, (int64_t*)p, ws, 8, nullptr, nullptr) == SC_ENOMEM);
    EXPECT(sc_remove_seam(p, 4, 4, 3, 11, (int32_t*)p, nullptr) == SC_EINVAL);
    EXPECT(sc_transpose_u8(p, 4, 4, 3, 12, p + 8, 12, nullptr) == SC_EINVAL);  // overlap
    EXPECT(sc_carve(p, 10, 10, 3, 11, 30, nullptr, nullptr, ws, big, nullptr, nullptr, nullptr) == SC_EINVAL);
    EXPECT(sc_carve(p, 10, 10, 3, 5, 30, nullptr, nullptr, fake + 1, big, nullptr, nullptr, nullptr) == SC_EINVAL);
    sc_tune bad = {1, 99, 0}, wide = {33, -1, 0};
    EXPECT(sc_carve(p, 10, 10, 3, 5, 30, nullptr, nullptr, ws, big, nullptr, nullptr, &bad) == SC_EINVAL);
    EXPECT(sc_carve(p, 10, 10, 3, 5, 30, nullptr, nullptr, ws, big, nullptr, nullptr, &wide) == SC_EUNSUPPORTED);
    EXPECT(sc_carve_noalloc(p, 4096, 4096, 3, 4000, 4096 * 3, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           SC_ENOMEM);
    EXPECT(sc_insert_seams(p, 10, 10, 3, 30, 10, p + 4096, 60, nullptr, nullptr, ws, big, nullptr) == SC_EINVAL);
    EXPECT(sc_insert_seams(p, 10, 10, 3, 30, 4, p + 100, 60, nullptr, nullptr, ws, big, nullptr) == SC_EINVAL);
    EXPECT(sc_carve_forward(p, 10, 9000, 3, 5, 27000, nullptr, nullptr, ws, big, nullptr, nullptr) ==
           SC_EUNSUPPORTED);
    sc_object_info info;
    EXPECT(sc_remove_object(p, p + 1000, 10, 10, 3, 30, 10, 2, 0, p + 2000, 30, &info, nullptr, nullptr, ws, big,
                            nullptr) == SC_EINVAL);
    EXPECT(sc_remove_object(p, p + 1000, 10, 10, 3, 30, 10, -1, 0, p + 10, 30, &info, nullptr, nullptr, ws, big,
                            nullptr) == SC_EINVAL);  // out overlaps img
    EXPECT(sc_remove_object(p, p + 1000, 10, 10, 3, 30, 10, -1, 0, p + 2000, 30, &info, nullptr, nullptr, ws, 64,
                            nullptr) == SC_ENOMEM);
    EXPECT(sc_slot_clear(p, 4, 4, nullptr) == SC_EINVAL && sc_slot_clear(p, 4, -1, nullptr) == SC_EINVAL);
    EXPECT(sc_slots_step_timed(p, 0, 1, 0, nullptr, nullptr) == SC_EINVAL);

    // valid arguments: validation passes and the (stand-in) launch fails with SC_EHIP
    EXPECT(sc_energy(p, 5, 5, 3, 15, (int32_t*)p, nullptr) == SC_EHIP);
    EXPECT(sc_carve(p, 10, 10, 3, 5, 30, nullptr, nullptr, ws, big, nullptr, nullptr, nullptr) == SC_EHIP);
    EXPECT(sc_carve_forward(p, 10, 12, 3, 5, 36, nullptr, nullptr, ws, big, nullptr, nullptr) == SC_EHIP);
    EXPECT(sc_remove_object(p, p + 1000, 10, 10, 3, 30, 10, 0, 1, p + 2000, 30, &info, nullptr, nullptr, ws, big,
                            nullptr) == SC_EHIP);

    // the batch planner: many jobs of uneven size; the host plan is built before the upload,
    // which fails here (no device)
    std::vector<sc_job> jobs;
    uint64_t x = 88172645463325252ull;
    auto rnd = [&](int lo, int hi) {
        x ^= x << 13, x ^= x >> 7, x ^= x << 17;
        return lo + (int)(x % (uint64_t)(hi - lo + 1));
    };
    for (int i = 0; i < 300; ++i) {
        sc_job j{};
        j.img = p;
        j.H = rnd(1, 2160);
        j.W = rnd(1, 2160);
        j.C = rnd(1, 4);
        j.pitch = j.W * j.C + rnd(0, 64);
        j.target_w = rnd(1, j.W);
        j.src = (i % 3) ? p : nullptr;
        jobs.push_back(j);
    }
    const size_t need = sc_batch_workspace_bytes(jobs.data(), (int)jobs.size());
    EXPECT(need > 0);
    sc_batch_info bi;
    for (int team : {0, 1, 4, 16, 32}) {
        sc_tune tn = {team, -1, 0};
        const sc_status s = sc_batch_prepare(jobs.data(), (int)jobs.size(), &tn, ws, need, &bi);
        EXPECT(s == SC_EHIP || s == SC_OK);
    }
    EXPECT(sc_batch_prepare(jobs.data(), (int)jobs.size(), nullptr, ws, need - 1, &bi) == SC_ENOMEM);
    jobs[7].target_w = 0;
    EXPECT(sc_batch_prepare(jobs.data(), (int)jobs.size(), nullptr, ws, need, &bi) == SC_EINVAL);
    jobs[7].target_w = 1;
    const size_t fneed = sc_forward_batch_workspace_bytes(jobs.data(), (int)jobs.size());
    EXPECT(fneed > 0);
    const sc_status fs = sc_forward_batch_prepare(jobs.data(), (int)jobs.size(), ws, fneed, &bi);
    EXPECT(fs == SC_EHIP || fs == SC_OK);
    EXPECT(sc_last_error() != nullptr);

    if (g_fail) std::fprintf(stderr, "%d expectation(s) failed\n", g_fail);
    else std::printf("api driver: all expectations held\n");
    return g_fail ? 1 : 0;
}
