// C ABI of libseamcarve: argument validation, workspace layout, batch planning, launches.
// Declarations and the meaning of every argument: include/sc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "../../include/sc.h"
#include "sc_internal.h"

namespace {

thread_local char g_err[512] = "";

sc_status fail(sc_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

sc_status ok() {
    g_err[0] = 0;
    return SC_OK;
}

sc_status hip_fail(hipError_t e, const char* what) {
    return fail(SC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Workspace header: the first 256 bytes of every workspace, then one Ctl per image.
struct WsHead {
    uint32_t magic;
    int32_t n;
    uint32_t pad[62];
};
constexpr uint32_t kMagic = sc::kWsMagic;
static_assert(sizeof(WsHead) == sc::kWsHeadBytes, "header size");
static_assert(sizeof(sc::Ctl) == 128, "ctl size");
static_assert(sc::kWsImgOffset + sizeof(sc::Img) <= sc::kWsHeadBytes, "a single image's descriptor fits the header");

constexpr int kMaxCostBound = 8388000;  // H*510*C: the column cost must fit 23 bits
constexpr int kDefaultTeamSingle = 8;   // workgroups carving one image (sc_carve)
constexpr int kDefaultTeamBatch = 16;   // largest team for one image of a batch

sc_status check_image(int H, int W, int C, int pitch) {
    if (H < 1 || W < 1) return fail(SC_EINVAL, "H=%d W=%d must be >= 1", H, W);
    if (C < 1 || C > 4) return fail(SC_EINVAL, "C=%d must be in 1..4", C);
    if ((long long)pitch < (long long)W * C) return fail(SC_EINVAL, "pitch=%d < W*C=%lld", pitch, (long long)W * C);
    if (W > 65535) return fail(SC_EUNSUPPORTED, "W=%d > 65535", W);
    if ((long long)H * 510 * C > kMaxCostBound)
        return fail(SC_EUNSUPPORTED, "H*510*C=%lld exceeds %d (23-bit cumulative cost)", (long long)H * 510 * C,
                    kMaxCostBound);
    return SC_OK;
}

size_t ctl_region(int n) { return sc::align_up(sizeof(WsHead) + (size_t)n * sizeof(sc::Ctl), sc::kAlign); }

// Fill the device descriptor of one image whose scratch starts at `base` and whose Ctl is `ctl`.
sc::Img make_img(const uint8_t* src, uint8_t* img, int H, int W, int C, long long pitch, int target_w,
                 int32_t* seams_out, int64_t* costs_out, char* base, sc::Ctl* ctl, int kr, int G, int mode) {
    const sc::Layout L = sc::layout_for(H, W, C, 32);
    sc::Img d;
    memset(&d, 0, sizeof(d));
    d.src = src;
    d.img = img;
    d.pitch = pitch;
    d.H = H;
    d.W = W;
    d.C = C;
    d.target_w = target_w;
    d.seams_out = seams_out;
    d.costs_out = reinterpret_cast<long long*>(costs_out);
    d.e = reinterpret_cast<uint16_t*>(base + L.e);
    d.dirs = reinterpret_cast<uint8_t*>(base + L.dirs);
    d.anc = reinterpret_cast<int8_t*>(base + L.anc);
    d.xq = reinterpret_cast<uint32_t*>(base + L.xq);
    d.seam = reinterpret_cast<int32_t*>(base + L.seam);
    d.ro = reinterpret_cast<int32_t*>(base + L.ro);
    d.wk = reinterpret_cast<uint8_t*>(base + L.wk);
    d.wp = L.wp;
    d.minside = 1;
    d.amin = &ctl->amin;
    d.bar = &ctl->bar;
    d.status = &ctl->status;
    d.ep = L.ep;
    d.db = L.db;
    d.xw = L.xw;
    d.P = (H + kr - 1) / kr;
    d.G = G;
    d.mode = mode;
    return d;
}

int resolve_variant(const sc_tune* t) {
    if (t && t->variant >= 0) return t->variant < sc::variant_count() ? t->variant : -1;
    return sc::default_variant();
}

}  // namespace

namespace sc {

Layout layout_for(int H, int W, int C, int kr_min) {
    Layout L;
    const int P = (H + kr_min - 1) / kr_min;
    L.P = P;
    L.ep = (int)align_up((size_t)W + 8, 64);
    L.db = (int)align_up((size_t)(W + 3) / 4 + 4, 16);
    L.xw = (int)align_up((size_t)W + 16, 64);
    size_t off = 0;
    L.ctl = 0;
    L.e = off;
    off = align_up(off + (size_t)H * L.ep * 2, kAlign);
    L.dirs = off;
    off = align_up(off + (size_t)align_up((size_t)H, 4) * L.db, kAlign);  // rows grouped by four
    L.anc = off;
    off = align_up(off + (size_t)P * W, kAlign);
    L.xq = off;
    off = align_up(off + (size_t)2 * L.xw * 4, kAlign);
    L.seam = off;
    off = align_up(off + (size_t)H * 4, kAlign);
    L.ro = off;
    off = align_up(off + (size_t)H * 4, kAlign);
    // working image: 64-byte aligned rows, so a 16-byte slot never spans two rows
    L.wp = (int)align_up((size_t)W * C, 64);
    L.wk = off;
    off = align_up(off + (size_t)H * L.wp, kAlign);
    L.total = off + kAlign;  // slack: row copies read a few bytes past the last row
    return L;
}

}  // namespace sc

extern "C" {

const char* sc_last_error(void) { return g_err; }

const char* sc_version(void) { return "seamcarve-mi355x 0.1 (gfx950)"; }

int sc_variant_count(void) { return sc::variant_count(); }

const char* sc_variant_name(int v) {
    if (v < 0 || v >= sc::variant_count()) return "";
    return sc::variant(v).name;
}

size_t sc_workspace_bytes(int H, int W, int C) {
    if (H < 1 || W < 1 || C < 1 || C > 4) return 0;
    return ctl_region(1) + sc::layout_for(H, W, C, 32).total;
}

sc_status sc_energy(const uint8_t* img, int H, int W, int C, int pitch, int32_t* energy, void* stream) {
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (!img || !energy) return fail(SC_EINVAL, "null pointer");
    hipError_t e = sc::launch_energy_i32(img, H, W, C, pitch, energy, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    return ok();
}

sc_status sc_dp_seam(const int32_t* energy, int H, int W, int32_t* seam, int64_t* cost, void* ws, size_t ws_bytes,
                     void* stream, uint8_t* dirs_out) {
    sc_status s = check_image(H, W, 1, W);
    if (s != SC_OK) return s;
    if (!energy || !seam || !cost || !ws) return fail(SC_EINVAL, "null pointer");
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const size_t need = sc_workspace_bytes(H, W, 1);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    const int v = sc::default_variant();
    char* base = static_cast<char*>(ws);
    sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead));
    sc::Img d = make_img(nullptr, nullptr, H, W, 1, W, W > 1 ? W - 1 : 1, seam, cost, base + ctl_region(1), ctl,
                         sc::variant(v).kr, 1, 1);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = sc::launch_prepare_from_i32(d, energy, st);
    if (e == hipSuccess) e = sc::launch_carve_single(d, v, 1, 0, st);
    if (e == hipSuccess && dirs_out) e = sc::launch_unpack_dirs(d, dirs_out, st);
    if (e != hipSuccess) return hip_fail(e, "dp launch");
    return ok();
}

sc_status sc_remove_seam(uint8_t* img, int H, int W, int C, int pitch, const int32_t* seam, void* stream) {
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (!img || !seam) return fail(SC_EINVAL, "null pointer");
    hipError_t e = sc::launch_remove_seam(img, H, W, C, pitch, seam, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "remove launch");
    return ok();
}

sc_status sc_transpose_u8(const uint8_t* src, int H, int W, int C, int src_pitch, uint8_t* dst, int dst_pitch,
                          void* stream) {
    if (H < 1 || W < 1 || C < 1 || C > 4) return fail(SC_EINVAL, "bad shape H=%d W=%d C=%d", H, W, C);
    if ((long long)src_pitch < (long long)W * C || (long long)dst_pitch < (long long)H * C)
        return fail(SC_EINVAL, "pitch too small");
    if (!src || !dst) return fail(SC_EINVAL, "null pointer");
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (size_t)(H - 1) * src_pitch + (size_t)W * C;
    const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + (size_t)(W - 1) * dst_pitch + (size_t)H * C;
    if (s0 < d1 && d0 < s1) return fail(SC_EINVAL, "src and dst overlap");
    hipError_t e = sc::launch_transpose(src, H, W, C, src_pitch, dst, dst_pitch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "transpose launch");
    return ok();
}

sc_status sc_carve(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out, int64_t* costs_out,
                   void* ws, size_t ws_bytes, void* stream, const uint8_t* src, const sc_tune* tune) {
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (!img || !ws) return fail(SC_EINVAL, "null pointer");
    if (target_w < 1 || target_w > W) return fail(SC_EINVAL, "target_w=%d not in [1, W=%d]", target_w, W);
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const size_t need = sc_workspace_bytes(H, W, C);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    const int v = resolve_variant(tune);
    if (v < 0) return fail(SC_EINVAL, "unknown kernel variant %d", tune->variant);
    const int G = tune && tune->team > 0 ? tune->team : kDefaultTeamSingle;
    if (G > 32) return fail(SC_EUNSUPPORTED, "team of %d workgroups > 32", G);
    char* base = static_cast<char*>(ws);
    sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead));
    sc::Img d = make_img(src, img, H, W, C, pitch, target_w, seams_out, costs_out, base + ctl_region(1), ctl,
                         sc::variant(v).kr, G, 0);
    if (tune && (tune->flags & SC_TUNE_NO_MINSIDE)) d.minside = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = sc::launch_prepare_single(d, st);
    const int xcd = tune ? (tune->flags >> SC_TUNE_XCD_SHIFT) & 7 : 0;
    if (e == hipSuccess && target_w < W) e = sc::launch_carve_single(d, v, G, xcd, st);
    if (e != hipSuccess) return hip_fail(e, "carve launch");
    return ok();
}

// sc_carve with its scratch in the library's fixed per-GPU device array instead of a caller's
// workspace: same validation, same kernels, no allocation of any kind.
sc_status sc_carve_noalloc(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out,
                           int64_t* costs_out, uint32_t* status_out, void* stream, const uint8_t* src,
                           const sc_tune* tune) {
    static_assert(sc::kNoAllocScratchBytes == (size_t)SC_NOALLOC_SCRATCH_BYTES, "scratch size");
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    const size_t need = sc_workspace_bytes(H, W, C);
    if (need > sc::kNoAllocScratchBytes)
        return fail(SC_ENOMEM, "a %dx%dx%d image needs %zu bytes of scratch; the fixed scratch holds %zu", H, W, C,
                    need, sc::kNoAllocScratchBytes);
    if (!img) return fail(SC_EINVAL, "null pointer");
    if (target_w < 1 || target_w > W) return fail(SC_EINVAL, "target_w=%d not in [1, W=%d]", target_w, W);
    void* ws = nullptr;
    hipError_t e = sc::noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    s = sc_carve(img, H, W, C, target_w, pitch, seams_out, costs_out, ws, sc::kNoAllocScratchBytes, stream, src,
                 tune);
    if (s != SC_OK) return s;
    if (status_out) {
        const sc::Ctl* ctl = reinterpret_cast<const sc::Ctl*>(static_cast<const char*>(ws) + sizeof(WsHead));
        e = sc::launch_copy_status(&ctl->status, status_out, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "status copy");
    }
    return ok();
}

namespace {
// Workspace of sc_insert_seams: the carve's own workspace, a scratch image the carve writes, the
// seams in removal coordinates and in original columns, and the per-row Fenwick trees.
struct InsertLayout {
    size_t carve, scratch, cur, orig, tree, total;
};

InsertLayout insert_layout(int H, int W, int C, int pitch, int k) {
    InsertLayout L;
    size_t off = 0;
    L.carve = off;
    off = sc::align_up(off + sc_workspace_bytes(H, W, C), sc::kAlign);
    L.scratch = off;
    off = sc::align_up(off + (size_t)H * pitch, sc::kAlign);
    L.cur = off;
    off = sc::align_up(off + (size_t)std::max(k, 1) * H * 4, sc::kAlign);
    L.orig = off;
    off = sc::align_up(off + (size_t)std::max(k, 1) * H * 4, sc::kAlign);
    L.tree = off;
    off = sc::align_up(off + (size_t)(W + 1) * H * 4, sc::kAlign);
    L.total = off;
    return L;
}
}  // namespace

size_t sc_insert_workspace_bytes(int H, int W, int C, int pitch, int k) {
    if (H < 1 || W < 1 || C < 1 || C > 4 || pitch < W * C || k < 0 || k >= W) return 0;
    return insert_layout(H, W, C, pitch, k).total;
}

sc_status sc_insert_seams(const uint8_t* img, int H, int W, int C, int pitch, int k, uint8_t* out, int out_pitch,
                          int32_t* seams_out, const sc_tune* tune, void* ws, size_t ws_bytes, void* stream) {
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (!img || !out || !ws) return fail(SC_EINVAL, "null pointer");
    if (k < 0 || k >= W) return fail(SC_EINVAL, "k=%d not in [0, W=%d)", k, W);
    if (W > sc::kInsertMaxWidth) return fail(SC_EUNSUPPORTED, "W=%d > %d", W, sc::kInsertMaxWidth);
    if ((long long)out_pitch < (long long)(W + k) * C)
        return fail(SC_EINVAL, "out_pitch=%d < (W + k) * C = %lld", out_pitch, (long long)(W + k) * C);
    const uintptr_t a0 = (uintptr_t)img, a1 = a0 + (size_t)(H - 1) * pitch + (size_t)W * C;
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (size_t)(H - 1) * out_pitch + (size_t)(W + k) * C;
    if (a0 < b1 && b0 < a1) return fail(SC_EINVAL, "out overlaps img");
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const InsertLayout L = insert_layout(H, W, C, pitch, k);
    if (ws_bytes < L.total) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, L.total);
    char* base = static_cast<char*>(ws);
    int32_t* orig = seams_out ? seams_out : reinterpret_cast<int32_t*>(base + L.orig);
    hipStream_t st = (hipStream_t)stream;
    if (k > 0) {
        // the seams: carve a copy (img is the source and stays unmodified), recording each seam
        s = sc_carve(reinterpret_cast<uint8_t*>(base + L.scratch), H, W, C, W - k, pitch,
                     reinterpret_cast<int32_t*>(base + L.cur), nullptr, base + L.carve, sc_workspace_bytes(H, W, C),
                     stream, img, tune);
        if (s != SC_OK) return s;
        hipError_t e = sc::launch_seam_origins(reinterpret_cast<const int32_t*>(base + L.cur), k, H, W,
                                               reinterpret_cast<int32_t*>(base + L.tree), orig, st);
        if (e != hipSuccess) return hip_fail(e, "seam origins launch");
    }
    hipError_t e = sc::launch_insert_seams(img, H, W, C, pitch, k, orig, out, out_pitch, st);
    if (e != hipSuccess) return hip_fail(e, "insert launch");
    return ok();
}

size_t sc_batch_workspace_bytes(const sc_job* jobs, int n) {
    if (!jobs || n < 1) return 0;
    size_t total = ctl_region(n);
    total += sc::align_up((size_t)n * sizeof(sc::Img), sc::kAlign);
    // plan arrays: blocks (<= 8 * n * 32 int2), teams (n int2), team images (n int)
    total += sc::align_up((size_t)8 * 32 * n * sizeof(int2), sc::kAlign);
    total += sc::align_up((size_t)n * sizeof(int2), sc::kAlign);
    total += sc::align_up((size_t)n * sizeof(int), sc::kAlign);
    for (int i = 0; i < n; ++i) {
        if (jobs[i].H < 1 || jobs[i].W < 1) return 0;
        total += sc::layout_for(jobs[i].H, jobs[i].W, jobs[i].C, 32).total;
    }
    return total;
}

sc_status sc_batch_prepare(const sc_job* jobs, int n, const sc_tune* tune, void* ws, size_t ws_bytes,
                           sc_batch_info* info) {
    if (!jobs || n < 1 || !ws || !info) return fail(SC_EINVAL, "null pointer or n < 1");
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    for (int i = 0; i < n; ++i) {
        const sc_job& j = jobs[i];
        sc_status s = check_image(j.H, j.W, j.C, j.pitch);
        if (s != SC_OK) return fail(s, "job %d: %s", i, g_err);
        if (!j.img) return fail(SC_EINVAL, "job %d: null image", i);
        if (j.target_w < 1 || j.target_w > j.W) return fail(SC_EINVAL, "job %d: target_w=%d not in [1, %d]", i,
                                                            j.target_w, j.W);
    }
    const size_t need = sc_batch_workspace_bytes(jobs, n);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    const int v = resolve_variant(tune);
    if (v < 0) return fail(SC_EINVAL, "unknown kernel variant %d", tune->variant);
    int G = tune && tune->team > 0 ? tune->team : kDefaultTeamBatch;
    if (G > 32) return fail(SC_EUNSUPPORTED, "team of %d workgroups > 32", G);

    // work of every image: pixel-seams = sum over seams of the current image's pixels
    std::vector<double> work(n);
    for (int i = 0; i < n; ++i) {
        const double k = jobs[i].W - jobs[i].target_w;
        work[i] = (double)jobs[i].H * (k * jobs[i].W - k * (k - 1) / 2) + 1.0;
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });

    // Team sizes.  An image whose work exceeds the average work per workgroup slot gets a team
    // of up to G workgroups on one XCD (their blocks come first in the grid, so every team is
    // resident at once); every other image gets one workgroup, launched longest first so the
    // dispatcher hands the next image to whichever slot frees up.
    int dev = 0, ncu = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return hip_fail(he, "device query");
    const int per_cu = std::max(1, sc::carve_blocks_per_cu(v));
    const int per_xcd = per_cu * ncu / 8;
    double total = 0;
    for (double x : work) total += x;
    const double per_slot = total / std::max(1, per_cu * ncu);
    std::vector<int> gsz(n, 1);
    if (G > 1)
        for (int i = 0; i < n; ++i) gsz[i] = (int)std::min<double>(G, std::max(1.0, std::ceil(work[i] / per_slot)));
    // The image with the longest chain of seams x rows sets the batch time; it alone gets twice
    // the largest team (its removal and band work split over more waves), room permitting.
    if (G > 1 && n > 1) {
        int crit = 0;
        double cbest = -1;
        for (int i = 0; i < n; ++i) {
            const double c = (double)(jobs[i].W - jobs[i].target_w) * (jobs[i].H + 64);
            if (c > cbest) cbest = c, crit = i;
        }
        gsz[crit] = std::min(std::min(2 * G, 32), per_xcd);
    }
    std::vector<int2> blk, teams;
    std::vector<int> team_imgs;
    int slots[8] = {0};
    std::vector<std::pair<int, int2>> placed;
    int nb_team = 0;
    for (int i : order) {
        if (gsz[i] < 2) continue;
        // the XCD with the most free slots
        int x = 0;
        for (int c = 1; c < 8; ++c)
            if (slots[c] < slots[x]) x = c;
        if (slots[x] + gsz[i] > per_xcd) {
            gsz[i] = 1;  // no room for a resident team: carve it with one workgroup
            continue;
        }
        const int t = (int)teams.size();
        teams.push_back(make_int2((int)team_imgs.size(), 1));
        team_imgs.push_back(i);
        for (int r = 0; r < gsz[i]; ++r) {
            const int b = x + 8 * (slots[x] + r);
            placed.push_back({b, make_int2(t, r)});
            nb_team = std::max(nb_team, b + 1);
        }
        slots[x] += gsz[i];
    }
    blk.assign(nb_team, make_int2(-1, -1));
    for (auto& pr : placed) blk[pr.first] = pr.second;
    // one workgroup per remaining image, in order of decreasing chain (seams x rows): a single
    // workgroup's carve time follows its row chain more than its pixel work (a tall narrow image
    // has little work but a long chain), and the longest must start first
    std::vector<int> singles;
    for (int i : order)
        if (gsz[i] < 2) singles.push_back(i);
    std::stable_sort(singles.begin(), singles.end(), [&](int a, int b) {
        return (double)(jobs[a].W - jobs[a].target_w) * jobs[a].H > (double)(jobs[b].W - jobs[b].target_w) * jobs[b].H;
    });
    for (int i : singles) {
        const int t = (int)teams.size();
        teams.push_back(make_int2((int)team_imgs.size(), 1));
        team_imgs.push_back(i);
        blk.push_back(make_int2(t, 0));
    }

    // host image of the plan region
    const size_t off_imgs = ctl_region(n);
    const size_t off_blk = off_imgs + sc::align_up((size_t)n * sizeof(sc::Img), sc::kAlign);
    const size_t off_teams = off_blk + sc::align_up((size_t)8 * 32 * n * sizeof(int2), sc::kAlign);
    const size_t off_ti = off_teams + sc::align_up((size_t)n * sizeof(int2), sc::kAlign);
    size_t off_data = off_ti + sc::align_up((size_t)n * sizeof(int), sc::kAlign);
    if (blk.size() > (size_t)8 * 32 * n) return fail(SC_EUNSUPPORTED, "plan too large");
    int teams_used = 0;
    for (int i = 0; i < n; ++i) teams_used += gsz[i] > 1;
    std::vector<char> host(off_data, 0);
    WsHead* h = reinterpret_cast<WsHead*>(host.data());
    h->magic = kMagic;
    h->n = n;
    char* base = static_cast<char*>(ws);
    sc::Img* imgs = reinterpret_cast<sc::Img*>(host.data() + off_imgs);
    int max_rows = 1;
    for (int i = 0; i < n; ++i) {
        const sc_job& j = jobs[i];
        sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead)) + i;
        imgs[i] = make_img(j.src, j.img, j.H, j.W, j.C, j.pitch, j.target_w, j.seams_out, j.costs_out,
                           base + off_data, ctl, sc::variant(v).kr, gsz[i], 0);
        if (tune && (tune->flags & SC_TUNE_NO_MINSIDE)) imgs[i].minside = 0;
        off_data += sc::layout_for(j.H, j.W, j.C, 32).total;
        max_rows = std::max(max_rows, j.H);
    }
    memcpy(host.data() + off_blk, blk.data(), blk.size() * sizeof(int2));
    memcpy(host.data() + off_teams, teams.data(), teams.size() * sizeof(int2));
    memcpy(host.data() + off_ti, team_imgs.data(), team_imgs.size() * sizeof(int));
    hipError_t e = hipMemcpy(ws, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "plan upload");

    memset(info, 0, sizeof(*info));
    info->n = n;
    info->nblocks = (int)blk.size();
    info->variant = v;
    info->max_rows = max_rows;
    info->team = G;
    info->teams_used = teams_used;
    info->off_imgs = off_imgs;
    info->off_blk = off_blk;
    info->off_teams = off_teams;
    info->off_team_imgs = off_ti;
    return ok();
}

static sc_status batch_pass(const sc_batch_info* info, void* ws, void* stream, bool energy, bool carve) {
    if (!info || !ws || info->n < 1 || info->nblocks < 1 || info->team < 1) return fail(SC_EINVAL, "bad batch info");
    char* base = static_cast<char*>(ws);
    hipStream_t st = (hipStream_t)stream;
    const sc::Img* imgs = reinterpret_cast<const sc::Img*>(base + info->off_imgs);
    hipError_t e = hipSuccess;
    if (energy) e = sc::launch_prepare_batch(imgs, info->n, info->max_rows, st);
    if (e == hipSuccess && carve)
        e = sc::launch_carve_batch(imgs, reinterpret_cast<const int2*>(base + info->off_blk),
                                   reinterpret_cast<const int2*>(base + info->off_teams),
                                   reinterpret_cast<const int*>(base + info->off_team_imgs), info->nblocks,
                                   info->variant, st);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return ok();
}

sc_status sc_batch_launch(const sc_batch_info* info, void* ws, void* stream) {
    return batch_pass(info, ws, stream, true, true);
}

sc_status sc_batch_launch_energy(const sc_batch_info* info, void* ws, void* stream) {
    return batch_pass(info, ws, stream, true, false);
}

sc_status sc_batch_launch_carve(const sc_batch_info* info, void* ws, void* stream) {
    return batch_pass(info, ws, stream, false, true);
}

sc_status sc_carve_batch(const sc_job* jobs, int n, const sc_tune* tune, void* ws, size_t ws_bytes, void* stream) {
    sc_batch_info info;
    sc_status s = sc_batch_prepare(jobs, n, tune, ws, ws_bytes, &info);
    if (s != SC_OK) return s;
    return sc_batch_launch(&info, ws, stream);
}

int sc_read_status(const void* ws, uint32_t* flags, int max_n) {
    if (!ws || !flags || max_n < 1) {
        fail(SC_EINVAL, "bad arguments");
        return -1;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        fail(SC_EHIP, "device synchronize failed");
        return -1;
    }
    WsHead h;
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess || h.magic != kMagic || h.n < 1) {
        fail(SC_EINVAL, "not a prepared workspace");
        return -1;
    }
    const int n = std::min(h.n, max_n);
    std::vector<sc::Ctl> c(n);
    if (hipMemcpy(c.data(), static_cast<const char*>(ws) + sizeof(WsHead), n * sizeof(sc::Ctl),
                  hipMemcpyDeviceToHost) != hipSuccess) {
        fail(SC_EHIP, "status copy failed");
        return -1;
    }
    for (int i = 0; i < n; ++i) flags[i] = c[i].status;
    ok();
    return n;
}

}  // extern "C"

extern "C" int sc_read_times(const void* ws, uint64_t* t_begin, uint64_t* t_end, int max_n, double* hz) {
    if (!ws || !t_begin || !t_end || max_n < 1) {
        fail(SC_EINVAL, "bad arguments");
        return -1;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        fail(SC_EHIP, "device synchronize failed");
        return -1;
    }
    WsHead h;
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess || h.magic != kMagic || h.n < 1) {
        fail(SC_EINVAL, "not a prepared workspace");
        return -1;
    }
    const int n = std::min(h.n, max_n);
    std::vector<sc::Ctl> c(n);
    if (hipMemcpy(c.data(), static_cast<const char*>(ws) + sizeof(WsHead), n * sizeof(sc::Ctl),
                  hipMemcpyDeviceToHost) != hipSuccess) {
        fail(SC_EHIP, "times copy failed");
        return -1;
    }
    for (int i = 0; i < n; ++i) {
        t_begin[i] = c[i].t_begin;
        t_end[i] = c[i].t_end;
    }
    if (hz) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            *hz = khz * 1000.0;
        else
            *hz = 100e6;
    }
    ok();
    return n;
}

extern "C" int sc_read_stages(const void* ws, uint64_t* stages, int max_n) {
    if (!ws || !stages || max_n < 1) {
        fail(SC_EINVAL, "bad arguments");
        return -1;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        fail(SC_EHIP, "device synchronize failed");
        return -1;
    }
    WsHead h;
    if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess || h.magic != kMagic || h.n < 1) {
        fail(SC_EINVAL, "not a prepared workspace");
        return -1;
    }
    const int n = std::min(h.n, max_n);
    std::vector<sc::Ctl> c(n);
    if (hipMemcpy(c.data(), static_cast<const char*>(ws) + sizeof(WsHead), n * sizeof(sc::Ctl),
                  hipMemcpyDeviceToHost) != hipSuccess) {
        fail(SC_EHIP, "stages copy failed");
        return -1;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 3; ++j) stages[3 * i + j] = c[i].t_stage[j];
    ok();
    return n;
}

// ---------------------------------------------------------------------------------- serving slots
constexpr size_t kSlotBytes = sizeof(sc::Img);  // the table is a device array of descriptors
constexpr int kMaxSlotTeam = 32;                // workgroups of one slot's team in a step

// The table: the slots' descriptors, then room for the block plan of a step with teams (teams
// laid out per XCD, then one block per slot).
size_t slot_plan_offset(int n_slots) { return sc::align_up((size_t)n_slots * kSlotBytes, sc::kAlign); }
size_t slot_plan_capacity(int n_slots) { return (size_t)8 * kMaxSlotTeam * n_slots + n_slots; }

extern "C" size_t sc_slot_table_bytes(int n_slots) {
    if (n_slots < 1) return 0;
    return slot_plan_offset(n_slots) + sc::align_up(slot_plan_capacity(n_slots) * sizeof(int4), sc::kAlign);
}

extern "C" sc_status sc_slot_start(const sc_job* job, void* ws, size_t ws_bytes, void* table, int n_slots, int slot,
                                   void* stream) {
    if (!job || !ws || !table) return fail(SC_EINVAL, "null pointer");
    if (n_slots < 1 || slot < 0 || slot >= n_slots) return fail(SC_EINVAL, "slot %d not in [0, %d)", slot, n_slots);
    sc_status s = check_image(job->H, job->W, job->C, job->pitch);
    if (s != SC_OK) return s;
    if (!job->img) return fail(SC_EINVAL, "null image");
    if (job->target_w < 1 || job->target_w > job->W)
        return fail(SC_EINVAL, "target_w=%d not in [1, W=%d]", job->target_w, job->W);
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const size_t need = sc_workspace_bytes(job->H, job->W, job->C);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    const int v = sc::default_variant();
    char* base = static_cast<char*>(ws);
    sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead));
    sc::Img d = make_img(job->src, job->img, job->H, job->W, job->C, job->pitch, job->target_w, job->seams_out,
                         job->costs_out, base + ctl_region(1), ctl, sc::variant(v).kr, 1, 0);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = sc::launch_prepare_single(d, st);
    if (e == hipSuccess) e = sc::launch_slot_write(static_cast<sc::Img*>(table), slot, d, st);
    if (e != hipSuccess) return hip_fail(e, "slot start");
    return ok();
}

extern "C" sc_status sc_slot_clear(void* table, int n_slots, int slot, void* stream) {
    if (!table) return fail(SC_EINVAL, "null table");
    if (n_slots < 1 || slot < 0 || slot >= n_slots) return fail(SC_EINVAL, "slot %d not in [0, %d)", slot, n_slots);
    sc::Img d;
    memset(&d, 0, sizeof(d));
    hipError_t e = sc::launch_slot_write(static_cast<sc::Img*>(table), slot, d, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "slot clear");
    return ok();
}

extern "C" sc_status sc_slots_step(const void* table, int n_slots, int max_seams, int32_t* progress, void* stream) {
    return sc_slots_step_timed(table, n_slots, max_seams, 0, progress, stream);
}

extern "C" sc_status sc_slots_step_timed(const void* table, int n_slots, int max_seams, long long budget_us,
                                         int32_t* progress, void* stream) {
    if (!table || n_slots < 1 || max_seams < 1 || budget_us < 0) return fail(SC_EINVAL, "bad slot step arguments");
    // the device wall clock runs at 100 MHz: 100 ticks per microsecond
    hipError_t e = sc::launch_carve_steps(static_cast<const sc::Img*>(table), n_slots, sc::default_variant(),
                                          max_seams, (unsigned long long)budget_us * 100ull, progress, nullptr, 0,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "slot step");
    return ok();
}

extern "C" sc_status sc_slots_step_teams(const void* table, int table_slots, int n_slots, const int32_t* team,
                                         int max_seams, long long budget_us, int32_t* progress, void* stream) {
    if (!table || !team || n_slots < 1 || max_seams < 1 || budget_us < 0)
        return fail(SC_EINVAL, "bad slot step arguments");
    if (table_slots < n_slots) return fail(SC_EINVAL, "n_slots=%d > table_slots=%d", n_slots, table_slots);
    const int v = sc::default_variant();
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    // Teams first in the grid, each on one XCD, all of them resident at once (their members wait
    // for each other); a team that finds no room carves with one workgroup.  Then one block per
    // remaining slot (those need no company and may wait for a free slot of the device).
    const int per_xcd = std::max(1, sc::carve_blocks_per_cu(v) * ncu / 8 * 3 / 4);
    std::vector<int> order;
    for (int s = 0; s < n_slots; ++s)
        if (team[s] > 1) order.push_back(s);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return team[a] > team[b]; });
    int used[8] = {0};
    std::vector<int4> plan;
    std::vector<char> single(n_slots, 1);
    for (int s : order) {
        const int G = std::min(team[s], kMaxSlotTeam);
        int x = 0;
        for (int c = 1; c < 8; ++c)
            if (used[c] < used[x]) x = c;
        if (used[x] + G > per_xcd) continue;
        for (int r = 0; r < G; ++r) {
            const size_t b = (size_t)x + 8 * (size_t)(used[x] + r);
            if (plan.size() <= b) plan.resize(b + 1, make_int4(-1, 0, 0, 0));
            plan[b] = make_int4(s, r, G, 0);
        }
        used[x] += G;
        single[s] = 0;
    }
    for (int s = 0; s < n_slots; ++s)
        if (single[s]) plan.push_back(make_int4(s, 0, 1, 0));
    if (plan.size() > slot_plan_capacity(table_slots)) return fail(SC_EUNSUPPORTED, "step plan too large");
    hipStream_t st = (hipStream_t)stream;
    char* base = static_cast<char*>(const_cast<void*>(table));
    // the plan goes after the descriptors of every slot of the table, so no descriptor is touched
    int4* dplan = reinterpret_cast<int4*>(base + slot_plan_offset(table_slots));
    e = hipMemcpyAsync(dplan, plan.data(), plan.size() * sizeof(int4), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = sc::launch_carve_steps(static_cast<const sc::Img*>(table), n_slots, v, max_seams,
                                   (unsigned long long)budget_us * 100ull, progress, dplan, (int)plan.size(), st);
    if (e != hipSuccess) return hip_fail(e, "slot step");
    return ok();
}

// ---------------------------------------------------------------------------------------------
// Forward energy (sec. "Forward Energy Calculation"): teams of 256-thread workgroups on one XCD,
// a dword per working pixel, no energy plane.
namespace {

struct FwdLayout {
    size_t dirs, anc, xq, amk, wk, total;
    int db, wp, xw, P;
};

FwdLayout fwd_layout(int H, int W, int C) {
    (void)C;
    FwdLayout L;
    L.P = (H + sc::kFwtPhaseRows - 1) / sc::kFwtPhaseRows;
    L.db = (int)sc::align_up((size_t)(W + 3) / 4, 16);  // direction bytes (4 columns each) per row
    L.wp = (int)sc::align_up((size_t)(W + 1) * 4, 64);   // one dword per pixel, and a copy of the last
    L.xw = (int)sc::align_up((size_t)W + 8, 64);
    size_t off = 0;
    L.dirs = off;
    off = sc::align_up(off + (size_t)((H + 3) / 4) * L.db * 4, sc::kAlign);  // rows grouped by four
    L.anc = off;
    off = sc::align_up(off + (size_t)L.P * W, sc::kAlign);
    L.xq = off;
    off = sc::align_up(off + (size_t)2 * L.xw * 4, sc::kAlign);
    L.amk = off;
    off = sc::align_up(off + 2 * sizeof(unsigned long long), sc::kAlign);
    L.wk = off;
    off = sc::align_up(off + (size_t)H * L.wp + sc::kFwdSlack, sc::kAlign);
    L.total = off;
    return L;
}

sc_status check_fwd_image(int H, int W, int C, int pitch) {
    sc_status s = check_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (W > sc::kFwdMaxW) return fail(SC_EUNSUPPORTED, "W=%d > %d (forward energy)", W, sc::kFwdMaxW);
    if (H > sc::kFwdMaxH) return fail(SC_EUNSUPPORTED, "H=%d > %d (forward energy)", H, sc::kFwdMaxH);
    if ((long long)H * (long long)sc::align_up((size_t)W * 4, 64) + (long long)sc::kFwdSlack >= (1ll << 31))
        return fail(SC_EUNSUPPORTED, "image of %lld pixels too large for the forward-energy path", (long long)H * W);
    return SC_OK;
}

// DP members of a forward team (the members whose windows cover the columns) and the team size
// whose waves (four per member) each walk and remove at most 4/rows_per_wave_phases phases of
// rows (half a phase by default).
int fwd_dp_members(int W) { return W <= sc::kFwtSingle ? 1 : (W + sc::kFwtOwned - 1) / sc::kFwtOwned; }
int fwd_team_target(int H, int W, int rows_per_wave_phases = 2) {
    const int P = (H + sc::kFwtPhaseRows - 1) / sc::kFwtPhaseRows;
    return std::min(32, std::max(fwd_dp_members(W), (P + rows_per_wave_phases - 1) / rows_per_wave_phases));
}
// A single image has the device to itself: its team grows until every wave walks and removes
// about 8 rows (measured at 1920x1080: 97 ms with 32 workgroups, 99 ms with 20, 109 ms with 10).
int fwd_single_team(int H, int W) { return std::min(32, std::max(fwd_dp_members(W), (H + 31) / 32)); }

sc::Img make_fwd_img(const uint8_t* src, uint8_t* img, int H, int W, int C, long long pitch, int target_w,
                     int32_t* seams_out, int64_t* costs_out, char* base, sc::Ctl* ctl, int G) {
    const FwdLayout L = fwd_layout(H, W, C);
    sc::Img d;
    memset(&d, 0, sizeof(d));
    d.src = src;
    d.img = img;
    d.pitch = pitch;
    d.H = H;
    d.W = W;
    d.C = C;
    d.target_w = target_w;
    d.seams_out = seams_out;
    d.costs_out = reinterpret_cast<long long*>(costs_out);
    d.dirs = reinterpret_cast<uint8_t*>(base + L.dirs);
    d.anc = reinterpret_cast<int8_t*>(base + L.anc);
    d.xq = reinterpret_cast<uint32_t*>(base + L.xq);
    d.xw = L.xw;
    d.amk = reinterpret_cast<unsigned long long*>(base + L.amk);
    d.wk = reinterpret_cast<uint8_t*>(base + L.wk);
    d.wp = L.wp;
    d.db = L.db;
    d.P = L.P;
    d.amin = &ctl->amin;
    d.bar = &ctl->bar;
    d.status = &ctl->status;
    d.G = G;
    return d;
}

double fwd_work(const sc_job& j) {  // pixel-seams: rows times the widths the seams are taken from
    const double k = j.W - j.target_w;
    return (double)j.H * k * (j.W + j.target_w + 1) / 2.0;
}

}  // namespace

extern "C" size_t sc_forward_workspace_bytes(int H, int W, int C) {
    if (H < 1 || W < 1 || C < 1 || C > 4) return 0;
    return ctl_region(1) + sc::align_up(sizeof(sc::Img), sc::kAlign) + fwd_layout(H, W, C).total;
}

extern "C" sc_status sc_carve_forward(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out,
                                      int64_t* costs_out, void* ws, size_t ws_bytes, void* stream, const uint8_t* src) {
    sc_status s = check_fwd_image(H, W, C, pitch);
    if (s != SC_OK) return s;
    if (!img || !ws) return fail(SC_EINVAL, "null pointer");
    if (target_w < 1 || target_w > W) return fail(SC_EINVAL, "target_w=%d not in [1, W=%d]", target_w, W);
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const size_t need = sc_forward_workspace_bytes(H, W, C);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    char* base = static_cast<char*>(ws);
    sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead));
    const size_t off_img = ctl_region(1);
    const int G = fwd_single_team(H, W);
    const sc::Img d = make_fwd_img(src, img, H, W, C, pitch, target_w, seams_out, costs_out,
                                   base + off_img + sc::align_up(sizeof(sc::Img), sc::kAlign), ctl, G);
    // header (magic, one image) and the descriptor, which the kernels read from the workspace
    WsHead h;
    memset(&h, 0, sizeof(h));
    h.magic = kMagic;
    h.n = 1;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(base, &h, sizeof(h), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(base + off_img, &d, sizeof(d), hipMemcpyHostToDevice, st);
    const sc::Img* dd = reinterpret_cast<const sc::Img*>(base + off_img);
    if (e == hipSuccess) e = sc::launch_fwt_prepare(dd, 1, H, st);
    if (e == hipSuccess && target_w < W) e = sc::launch_fwt_carve(dd, nullptr, 8 * G, 0, st);
    if (e != hipSuccess) return hip_fail(e, "forward carve launch");
    return ok();
}

extern "C" size_t sc_forward_batch_workspace_bytes(const sc_job* jobs, int n) {
    if (!jobs || n < 1) return 0;
    size_t total = ctl_region(n);
    total += sc::align_up((size_t)n * sizeof(sc::Img), sc::kAlign);
    total += sc::align_up((size_t)8 * 32 * n * sizeof(int2), sc::kAlign);
    for (int i = 0; i < n; ++i) {
        if (jobs[i].H < 1 || jobs[i].W < 1 || jobs[i].C < 1 || jobs[i].C > 4) return 0;
        total += fwd_layout(jobs[i].H, jobs[i].W, jobs[i].C).total;
    }
    return total;
}

extern "C" sc_status sc_forward_batch_prepare(const sc_job* jobs, int n, void* ws, size_t ws_bytes,
                                              sc_batch_info* info) {
    if (!jobs || n < 1 || !ws || !info) return fail(SC_EINVAL, "null pointer or n < 1");
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    int max_rows = 1;
    for (int i = 0; i < n; ++i) {
        const sc_job& j = jobs[i];
        sc_status s = check_fwd_image(j.H, j.W, j.C, j.pitch);
        if (s != SC_OK) return fail(s, "job %d: %s", i, g_err);
        if (!j.img) return fail(SC_EINVAL, "job %d: null image", i);
        if (j.target_w < 1 || j.target_w > j.W)
            return fail(SC_EINVAL, "job %d: target_w=%d not in [1, %d]", i, j.target_w, j.W);
        max_rows = std::max(max_rows, j.H);
    }
    const size_t need = sc_forward_batch_workspace_bytes(jobs, n);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);

    // Teams.  Every team's workgroups must be resident at once on one XCD (they wait for each
    // other), so the whole plan fits the device's resident workgroups: every image first gets its
    // DP members, then images in order of decreasing work grow toward a team in which every wave
    // walks and removes at most one phase of rows.
    int dev = 0, ncu = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return hip_fail(he, "device query");
    // two thirds of the occupancy the runtime reports: a plan that needed every last slot could
    // leave a team partly resident behind others (measured: planning for 3 workgroups per compute
    // unit made teams wait out their barriers)
    const int per_xcd = std::max(1, 2 * sc::fwt_blocks_per_cu() * ncu / 3 / 8);
    std::vector<int> order(n), gsz(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fwd_work(jobs[a]) > fwd_work(jobs[b]); });
    long long used = 0;
    for (int i = 0; i < n; ++i) used += gsz[i] = fwd_dp_members(jobs[i].W);
    const long long cap = 8ll * per_xcd;
    if (used > cap)
        return fail(SC_EUNSUPPORTED, "%lld workgroups of forward teams exceed the %lld resident ones; split the batch",
                    used, cap);
    // grow the teams while room is left: the image with the most work first toward half a phase of
    // rows per wave (it sets the batch time), then every image toward a phase per wave, then toward
    // half a phase, longest first
    auto grow_to = [&](int i, int per) {
        const int grow = std::min<long long>(fwd_team_target(jobs[i].H, jobs[i].W, per) - gsz[i], cap - used);
        if (grow > 0) gsz[i] += grow, used += grow;
    };
    grow_to(order[0], 2);
    for (int per : {4, 2})
        for (int i : order) grow_to(i, per);
    // placement: longest first, each team on the XCD with the most free slots
    int slots[8] = {0};
    std::vector<int2> blk;
    for (int i : order) {
        int x = 0;
        for (int c = 1; c < 8; ++c)
            if (slots[c] < slots[x]) x = c;
        while (slots[x] + gsz[i] > per_xcd && gsz[i] > fwd_dp_members(jobs[i].W)) --gsz[i];
        if (slots[x] + gsz[i] > per_xcd) return fail(SC_EUNSUPPORTED, "no XCD has room for the team of job %d", i);
        for (int r = 0; r < gsz[i]; ++r) {
            const size_t b = (size_t)x + 8 * (size_t)(slots[x] + r);
            if (blk.size() <= b) blk.resize(b + 1, make_int2(-1, -1));
            blk[b] = make_int2(i, r);
        }
        slots[x] += gsz[i];
    }
    if (blk.size() > (size_t)8 * 32 * n) return fail(SC_EUNSUPPORTED, "plan too large");
    const size_t off_imgs = ctl_region(n);
    const size_t off_blk = off_imgs + sc::align_up((size_t)n * sizeof(sc::Img), sc::kAlign);
    size_t off_data = off_blk + sc::align_up((size_t)8 * 32 * n * sizeof(int2), sc::kAlign);
    std::vector<char> host(off_data, 0);
    WsHead* h = reinterpret_cast<WsHead*>(host.data());
    h->magic = kMagic;
    h->n = n;
    char* base = static_cast<char*>(ws);
    sc::Img* imgs = reinterpret_cast<sc::Img*>(host.data() + off_imgs);
    for (int i = 0; i < n; ++i) {
        const sc_job& j = jobs[i];
        sc::Ctl* ctl = reinterpret_cast<sc::Ctl*>(base + sizeof(WsHead)) + i;
        imgs[i] = make_fwd_img(j.src, j.img, j.H, j.W, j.C, j.pitch, j.target_w, j.seams_out, j.costs_out,
                               base + off_data, ctl, gsz[i]);
        off_data += fwd_layout(j.H, j.W, j.C).total;
    }
    memcpy(host.data() + off_blk, blk.data(), blk.size() * sizeof(int2));
    hipError_t e = hipMemcpy(ws, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "forward batch upload");
    int teams = 0;
    for (int i = 0; i < n; ++i) teams += gsz[i] > 1;
    memset(info, 0, sizeof(*info));
    info->n = n;
    info->nblocks = (int)blk.size();
    info->variant = -1;     // the forward kernel has one shape
    info->max_rows = max_rows;
    info->team = 0;         // marks a forward-energy batch
    info->teams_used = teams;
    info->off_imgs = off_imgs;
    info->off_blk = off_blk;
    return ok();
}

static sc_status fwd_batch_pass(const sc_batch_info* info, void* ws, void* stream, bool copy, bool carve) {
    if (!info || !ws || info->n < 1 || info->nblocks < 1 || info->team != 0 || info->variant != -1)
        return fail(SC_EINVAL, "not a forward-energy batch");
    char* base = static_cast<char*>(ws);
    const sc::Img* imgs = reinterpret_cast<const sc::Img*>(base + info->off_imgs);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (copy) e = sc::launch_fwt_prepare(imgs, info->n, info->max_rows, st);
    if (e == hipSuccess && carve)
        e = sc::launch_fwt_carve(imgs, reinterpret_cast<const int2*>(base + info->off_blk), info->nblocks, 0, st);
    if (e != hipSuccess) return hip_fail(e, "forward batch launch");
    return ok();
}

extern "C" sc_status sc_forward_batch_launch(const sc_batch_info* info, void* ws, void* stream) {
    return fwd_batch_pass(info, ws, stream, true, true);
}

extern "C" sc_status sc_forward_batch_launch_copy(const sc_batch_info* info, void* ws, void* stream) {
    return fwd_batch_pass(info, ws, stream, true, false);
}

extern "C" sc_status sc_forward_batch_launch_carve(const sc_batch_info* info, void* ws, void* stream) {
    return fwd_batch_pass(info, ws, stream, false, true);
}

// ---------------------------------------------------------------------------------------------
// Object removal with a mask (sec. "Object Removal"): direction from the mask's extent, masked
// carve of the frame (the image, or its transpose for horizontal seams), optional restore by
// seam insertion, then the result back in the caller's orientation.
namespace {

struct ObjLayout {
    size_t ctl, desc, wk, mk, dirs, anc, seam, buf_a, buf_b, ins, ins_bytes, total;
    int wp, mp, db;
};

// Workspace of one carved frame of h rows by w0 columns.
ObjLayout obj_layout(int h, int w0, int C, bool restore) {
    ObjLayout L;
    const int P = (h + sc::kFwdPhaseRows - 1) / sc::kFwdPhaseRows;
    L.wp = (int)sc::align_up((size_t)w0 * C, 64);
    L.mp = (int)sc::align_up((size_t)w0, 64);
    L.db = (int)sc::align_up((size_t)(w0 + 3) / 4, 16);
    size_t off = 0;
    L.ctl = off;
    off = sc::align_up(off + sizeof(sc::ObjCtl), sc::kAlign);
    L.desc = off;
    off = sc::align_up(off + sizeof(sc::ObjImg), sc::kAlign);
    L.wk = off;
    off = sc::align_up(off + (size_t)h * L.wp + sc::kFwdSlack, sc::kAlign);
    L.mk = off;
    off = sc::align_up(off + (size_t)h * L.mp + sc::kFwdSlack, sc::kAlign);
    L.dirs = off;
    off = sc::align_up(off + (size_t)((h + 3) / 4) * L.db * 4, sc::kAlign);
    L.anc = off;
    off = sc::align_up(off + (size_t)P * w0, sc::kAlign);
    L.seam = off;
    off = sc::align_up(off + (size_t)h * 4, sc::kAlign);
    L.buf_a = L.buf_b = L.ins = L.ins_bytes = 0;
    if (restore && w0 >= 2) {
        L.buf_a = off;
        off = sc::align_up(off + (size_t)h * L.wp, sc::kAlign);
        L.buf_b = off;
        off = sc::align_up(off + (size_t)h * L.wp, sc::kAlign);
        L.ins = off;
        L.ins_bytes = sc_insert_workspace_bytes(h, w0, C, L.wp, w0 - 1);  // the largest round
        off = sc::align_up(off + L.ins_bytes, sc::kAlign);
    }
    L.total = off;
    return L;
}

sc_status check_obj_frame(int h, int w0, int C) {
    if (w0 > sc::kFwdMaxW) return fail(SC_EUNSUPPORTED, "%d columns to carve > %d", w0, sc::kFwdMaxW);
    if (h > sc::kFwdMaxH) return fail(SC_EUNSUPPORTED, "%d rows to carve > %d", h, sc::kFwdMaxH);
    if ((long long)h * 510 * C > kMaxCostBound)
        return fail(SC_EUNSUPPORTED, "rows*510*C=%lld exceeds %d (23-bit seam energy)", (long long)h * 510 * C,
                    kMaxCostBound);
    if ((long long)h * (long long)sc::align_up((size_t)w0 * C, 64) + (long long)sc::kFwdSlack >= (1ll << 31))
        return fail(SC_EUNSUPPORTED, "frame of %lld bytes too large", (long long)h * w0 * C);
    return SC_OK;
}

bool ranges_overlap(const void* a, size_t a_len, const void* b, size_t b_len) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + b_len && b0 < a0 + a_len;
}

}  // namespace

extern "C" size_t sc_object_workspace_bytes(int H, int W, int C, int restore) {
    if (H < 1 || W < 1 || C < 1 || C > 4) return 0;
    return std::max(obj_layout(H, W, C, restore != 0).total, obj_layout(W, H, C, restore != 0).total);
}

extern "C" sc_status sc_remove_object(const uint8_t* img, const uint8_t* mask, int H, int W, int C, int pitch,
                                      int mpitch, int direction, int restore, uint8_t* out, int out_pitch,
                                      sc_object_info* info, int32_t* seams_out, int64_t* costs_out, void* ws,
                                      size_t ws_bytes, void* stream) {
    if (H < 1 || W < 1) return fail(SC_EINVAL, "H=%d W=%d must be >= 1", H, W);
    if (C < 1 || C > 4) return fail(SC_EINVAL, "C=%d must be in 1..4", C);
    if ((long long)pitch < (long long)W * C) return fail(SC_EINVAL, "pitch=%d < W*C=%lld", pitch, (long long)W * C);
    if (mpitch < W) return fail(SC_EINVAL, "mpitch=%d < W=%d", mpitch, W);
    if ((long long)out_pitch < (long long)W * C)
        return fail(SC_EINVAL, "out_pitch=%d < W*C=%lld", out_pitch, (long long)W * C);
    if (direction < SC_OBJ_AUTO || direction > SC_OBJ_HORIZONTAL)
        return fail(SC_EINVAL, "direction=%d not in {-1, 0, 1}", direction);
    if (restore != 0 && restore != 1) return fail(SC_EINVAL, "restore=%d not 0 or 1", restore);
    if (!img || !mask || !out || !info || !ws) return fail(SC_EINVAL, "null pointer");
    const size_t img_len = (size_t)(H - 1) * pitch + (size_t)W * C;
    const size_t out_len = (size_t)(H - 1) * out_pitch + (size_t)W * C;
    if (ranges_overlap(out, out_len, img, img_len) || ranges_overlap(out, out_len, mask, (size_t)(H - 1) * mpitch + W))
        return fail(SC_EINVAL, "out overlaps img or mask");
    if ((uintptr_t)ws % sc::kAlign) return fail(SC_EINVAL, "workspace must be %zu-byte aligned", sc::kAlign);
    const size_t need = sc_object_workspace_bytes(H, W, C, restore);
    if (ws_bytes < need) return fail(SC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);
    sc::ObjCtl* ctl = reinterpret_cast<sc::ObjCtl*>(base);  // the control block sits first in both layouts
    sc::ObjCtl hc;
    hipError_t e = sc::launch_obj_reset(ctl, 1, st);
    if (e != hipSuccess) return hip_fail(e, "object reset");

    // the direction (synchronous: the frame to carve depends on it)
    int dir = direction;
    if (dir == SC_OBJ_AUTO) {
        e = sc::launch_mask_bbox(mask, H, W, mpitch, ctl->bbox, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "mask extent");
        const int r0 = hc.bbox[0], r1 = hc.bbox[1], c0 = hc.bbox[2], c1 = hc.bbox[3];
        dir = (r1 < 0 || (c1 - c0 + 1) <= (r1 - r0 + 1)) ? SC_OBJ_VERTICAL : SC_OBJ_HORIZONTAL;
    }
    const bool vert = dir == SC_OBJ_VERTICAL;
    const int h = vert ? H : W, w0 = vert ? W : H;
    sc_status s = check_obj_frame(h, w0, C);
    if (s != SC_OK) return s;
    const ObjLayout L = obj_layout(h, w0, C, restore != 0);
    uint8_t* wk = reinterpret_cast<uint8_t*>(base + L.wk);
    uint8_t* mk = reinterpret_cast<uint8_t*>(base + L.mk);

    // the frame: image and mask, copied or transposed into the working buffers
    if (vert) {
        e = sc::launch_copy_rows(img, pitch, wk, L.wp, H, W * C, st);
        if (e == hipSuccess) e = sc::launch_copy_rows(mask, mpitch, mk, L.mp, H, W, st);
    } else {
        e = sc::launch_transpose(img, H, W, C, pitch, wk, L.wp, st);
        if (e == hipSuccess) e = sc::launch_transpose(mask, H, W, 1, mpitch, mk, L.mp, st);
    }
    if (e != hipSuccess) return hip_fail(e, "object frame");

    // the masked carve: seams until the mask is gone (or one column is left)
    sc::ObjImg d;
    memset(&d, 0, sizeof(d));
    d.wk = wk;
    d.mk = mk;
    d.dirs = reinterpret_cast<uint8_t*>(base + L.dirs);
    d.anc = reinterpret_cast<int8_t*>(base + L.anc);
    d.seam = reinterpret_cast<int32_t*>(base + L.seam);
    d.seams_out = seams_out;
    d.costs_out = reinterpret_cast<long long*>(costs_out);
    d.ctl = ctl;
    d.out = nullptr;
    d.H = h;
    d.W = w0;
    d.C = C;
    d.wp = L.wp;
    d.mp = L.mp;
    d.db = L.db;
    d.max_seams = w0 - 1;
    sc::ObjImg* desc = reinterpret_cast<sc::ObjImg*>(base + L.desc);
    e = hipMemcpyAsync(desc, &d, sizeof(d), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = sc::launch_obj_carve(desc, 1, w0, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "object carve");
    const int k = hc.k, left = hc.left;
    int rw = hc.w;
    if (k < 0 || k > w0 - 1 || rw != w0 - k) return fail(SC_EHIP, "object carve returned k=%d w=%d", k, rw);

    // restore the size by seam insertion, in rounds of at most (current width - 1) seams
    const uint8_t* cur = wk;
    if (restore && k > 0) {
        if (rw < 2) return fail(SC_EINVAL, "the carve left one column: nothing to insert seams into");
        uint8_t* bufs[2] = {reinterpret_cast<uint8_t*>(base + L.buf_a), reinterpret_cast<uint8_t*>(base + L.buf_b)};
        int nb = 0;
        while (rw < w0) {
            const int n = std::min(w0 - rw, rw - 1);
            s = sc_insert_seams(cur, h, rw, C, L.wp, n, bufs[nb], L.wp, nullptr, nullptr, base + L.ins, L.ins_bytes,
                                stream);
            if (s != SC_OK) return s;
            cur = bufs[nb];
            nb ^= 1;
            rw += n;
        }
    }

    // the result in the caller's orientation
    if (vert) e = sc::launch_copy_rows(cur, L.wp, out, out_pitch, h, rw * C, st);
    else e = sc::launch_transpose(cur, h, rw, C, L.wp, out, out_pitch, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "object output");
    int dev = 0, khz = 0;
    double tick_ms = 0.0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        tick_ms = 1.0 / khz;
    memset(info, 0, sizeof(*info));
    info->direction = dir;
    info->k = k;
    info->rows = vert ? h : rw;
    info->cols = vert ? rw : h;
    info->left = left;
    info->carve_ms = (double)(hc.t_end - hc.t_begin) * tick_ms;
    for (int i = 0; i < 3; ++i) info->stage_ms[i] = (double)hc.t_stage[i] * tick_ms;
    return ok();
}
