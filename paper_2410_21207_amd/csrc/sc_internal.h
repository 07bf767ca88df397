// Internal structures of libseamcarve (not part of the C ABI).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sc {

// Device descriptor of one image being carved.  All pointers are device pointers.
struct Img {
    const uint8_t* src;  // optional source (else img is the source)
    uint8_t* img;        // H rows of `pitch` bytes: receives the carved image
    long long pitch;
    int H, W, C, target_w;
    int32_t* seams_out;  // optional, (W-target_w)*H
    long long* costs_out;  // optional, W-target_w
    // workspace pieces
    uint16_t* e;   // energy plane, H rows of `ep` uint16
    uint8_t* dirs; // parent directions, 2 bits per cell, H rows of `db` bytes
    int8_t* anc;   // per DP phase, the ancestor offset of every column at the phase's last row
    uint32_t* xq;  // 2 rows of `xw` uint32: DP keys exchanged between waves at phase ends
    int32_t* seam; // current seam, H
    int32_t* ro;   // per row: physical column of the row's first pixel (min-side removal), H
    uint8_t* wk;   // working copy of the image, H rows of `wp` bytes (64-byte aligned rows)
    unsigned long long* amin;  // packed (cost << 32 | column) argmin of the current seam
    unsigned* bar;             // team barrier counter
    unsigned* status;          // error bits
    int ep, db, xw, P;         // pitches and the number of DP phases
    int wp;                    // bytes per row of wk
    int G;                     // team size (workgroups) carving this image
    int mode;                  // 0 = carve, 1 = one seam only, no removal (sc_dp_seam)
    int minside;               // 1 = remove a seam pixel by moving the shorter side of its row
    unsigned long long* amk;   // forward teams: the argmin words of even and odd seams
};

// Control words of one image (zeroed by the energy pass of every launch).
struct Ctl {
    unsigned long long amin;            // packed (cost << 32 | column) argmin of the current seam
    unsigned bar;                       // team barrier counter
    unsigned status;                    // error bits (kStatus*)
    unsigned long long t_begin, t_end;  // device clock when the carve started / ended
    unsigned xmask;                     // XCDs the team's workgroups ran on (bit per XCD)
    unsigned done;                      // seams removed so far (step-wise carving)
    unsigned long long t_stage[3];      // device clock spent in: DP sweep; backtrack + removal; band update
    // step-wise carving by a team (serving): the barrier count the previous calls left, and the
    // stop decision of the team's first member at the end of a seam
    unsigned ebase;
    unsigned stop;
    unsigned pad[14];
};
constexpr unsigned kStatusTimeout = 1u;    // a team barrier timed out
constexpr unsigned kStatusPlacement = 2u;  // a team's workgroups were not on one XCD

// Placement of one image's scratch inside a workspace.
struct Layout {
    size_t ctl, e, dirs, anc, xq, seam, ro, wk, total;
    int ep, db, xw, P, wp;
};

constexpr size_t kAlign = 256;
constexpr uint32_t kWsMagic = 0x31574353u;  // "SCW1": first word of a prepared workspace
constexpr size_t kWsHeadBytes = 256;        // header, then one Ctl per image
constexpr size_t kWsImgOffset = 64;         // single-image workspaces keep their descriptor here
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Kernel variants: columns per lane, rows per DP phase, threads per workgroup.  X(id, cpl, kr,
// threads) for every compiled variant of the carve kernel; the launchers switch over the same list.
#define SC_VARIANTS(X)                                                                                      \
    X(0, 4, 32, 256) X(1, 4, 32, 512) X(2, 4, 32, 1024) X(3, 8, 32, 512) X(4, 8, 32, 1024) X(5, 4, 48, 512) \
    X(6, 4, 48, 256) X(7, 4, 56, 512) X(8, 4, 56, 256) X(9, 2, 48, 512)

struct Variant {
    int cpl, kr, threads;
    const char* name;
};
#define SC_VARIANT_ROW(id, c, k, t) {c, k, t, "cpl" #c "_k" #k "_t" #t},
inline constexpr Variant kVariants[] = {SC_VARIANTS(SC_VARIANT_ROW)};
#undef SC_VARIANT_ROW
inline int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
inline const Variant& variant(int v) { return kVariants[v]; }
inline int default_variant() { return 7; }  // cpl4_k56_t512

Layout layout_for(int H, int W, int C, int variant_kr_min);
constexpr int kLdsExchangeMaxW = 4096;  // single-workgroup carves keep the phase exchange row in LDS up to this width

// Launchers (sc_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_energy_i32(const uint8_t* img, int H, int W, int C, long long pitch, int32_t* out,
                             hipStream_t st);
hipError_t launch_prepare_single(const Img& d, hipStream_t st);          // energy plane (+copy, ctl zero)
hipError_t launch_prepare_from_i32(const Img& d, const int32_t* energy, hipStream_t st);
hipError_t launch_carve_single(const Img& d, int variant, int G, int xcd, hipStream_t st);
hipError_t launch_carve_steps(const Img* table, int n, int variant, int max_seams, unsigned long long budget_ticks,
                              int* progress, const int4* plan, int nblocks, hipStream_t st);
hipError_t launch_slot_write(Img* table, int slot, const Img& d, hipStream_t st);
hipError_t launch_unpack_dirs(const Img& d, uint8_t* out, hipStream_t st);
hipError_t launch_remove_seam(uint8_t* img, int H, int W, int C, long long pitch, const int32_t* seam,
                              hipStream_t st);
hipError_t launch_transpose(const uint8_t* src, int H, int W, int C, long long sp, uint8_t* dst, long long dp,
                            hipStream_t st);
hipError_t launch_prepare_batch(const Img* d_imgs, int n, int max_rows, hipStream_t st);
hipError_t launch_carve_batch(const Img* d_imgs, const int2* blk, const int2* teams, const int* team_imgs,
                              int nblocks, int variant, hipStream_t st);
int carve_blocks_per_cu(int variant);  // occupancy of the carve kernel
hipError_t launch_seam_origins(const int32_t* seams, int k, int H, int W, int32_t* tree, int32_t* orig,
                               hipStream_t st);
hipError_t launch_insert_seams(const uint8_t* img, int H, int W, int C, long long pitch, int k, const int32_t* orig,
                               uint8_t* out, long long out_pitch, hipStream_t st);
constexpr int kInsertMaxWidth = 65536;

// Limits of the one-workgroup-row kernels (object removal) and the forward teams: widths up to
// kFwdMaxW, rows up to kFwdMaxH; loads of a row may read up to kFwdSlack bytes past the last row of
// a working copy.  kFwdPhaseRows: rows per backtrack phase of the object-removal DP.
constexpr int kFwdMaxW = 8192;
constexpr int kFwdMaxH = 16448;
constexpr int kFwdPhaseRows = 60;
constexpr size_t kFwdSlack = 256;

// Forward-energy carve by teams of 256-thread workgroups on one XCD (sc_forward.hip).  A working
// pixel is one dword.  Member g of a team with more than one DP member computes columns
// [g*kFwtOwned - 2*kFwtPhaseRows, (g+1)*kFwtOwned + 2*kFwtPhaseRows) and owns [g*kFwtOwned,
// (g+1)*kFwtOwned); a team of images up to kFwtSingle columns has one DP member.  blk: block ->
// (image, member), or nullptr for one image whose members are blocks xcd, xcd + 8, ...
constexpr int kFwtThreads = 256;
constexpr int kFwtWindow = 976;  // 4 waves x 240 exact columns + 8 ghost columns on each side
constexpr int kFwtPhaseRows = 56;
constexpr int kFwtOwned = kFwtWindow - 4 * kFwtPhaseRows;  // keys exchanged every second phase
constexpr int kFwtSingle = kFwtWindow - 8;  // widest image a single DP member carves
hipError_t launch_fwt_prepare(const Img* imgs, int n, int max_rows, hipStream_t st);
hipError_t launch_fwt_carve(const Img* imgs, const int2* blk, int nblocks, int xcd, hipStream_t st);
int fwt_blocks_per_cu();

// Object removal with a mask (one 1024-thread workgroup per image, the forward kernel's limits:
// frame width <= kFwdMaxW, frame rows <= kFwdMaxH).  The carved frame is h = H rows by W columns
// (the transpose of the image for horizontal seams).
struct ObjCtl {
    int k;        // seams removed
    int left;     // masked pixels left when the carve stopped
    int w;        // columns left
    int bbox[4];  // mask bounding box: first row, last row, first column, last column
    int pad;
    unsigned long long t_begin, t_end;  // device clock when the carve started / ended
    unsigned long long t_stage[3];      // device clock in: DP sweep; argmin + backtrack; removal
};
struct ObjImg {
    uint8_t* wk;           // working image, H rows of wp bytes (64-byte aligned rows)
    uint8_t* mk;           // working mask, H rows of mp bytes (nonzero = masked)
    uint8_t* dirs;         // 2-bit direction map, rows grouped by four, db bytes per row group lane
    int8_t* anc;           // phase ancestors when they do not fit in LDS
    int32_t* seam;         // current seam, H
    int32_t* seams_out;    // optional, max_seams * H
    long long* costs_out;  // optional, max_seams
    ObjCtl* ctl;
    uint8_t* out;          // optional: the carved rows are copied here at the end
    long long out_pitch;
    int H, W, C, wp, mp, db, max_seams;
};
hipError_t launch_obj_reset(ObjCtl* ctl, int n, hipStream_t st);
hipError_t launch_obj_carve(const ObjImg* imgs, int n, int max_w, hipStream_t st);
hipError_t launch_mask_bbox(const uint8_t* mask, int H, int W, long long mpitch, int* bbox, hipStream_t st);
hipError_t launch_copy_rows(const uint8_t* src, long long sp, uint8_t* dst, long long dp, int rows, int bytes,
                            hipStream_t st);

// Allocation-free carve: the fixed device scratch of the current GPU (looked up once per device)
// and a one-thread copy of an image's status word to a caller's device word.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;  // = SC_NOALLOC_SCRATCH_BYTES of sc.h
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_copy_status(const unsigned* src, uint32_t* dst, hipStream_t st);

}  // namespace sc
