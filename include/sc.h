/*
 * sc.h -- C ABI of the MI355X seam-carving library (libseamcarve.so).
 *
 * Method: arXiv 2410.21207, "Analysis of Different Algorithmic Design
 * Techniques for Seam Carving".  The library runs the per-seam loop of that
 * paper on one gfx950 GPU: e1 gradient energy, the dynamic-programming
 * cumulative minimum-energy map M(i,j) = e(i,j) + min(M(i-1,j-1..j+1)), the
 * argmin of its last row, the backtrack, and the removal of the seam.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers owned by the caller unless a comment says
 *     "host".  The library never allocates or frees caller memory; every
 *     scratch buffer comes from the caller's workspace `ws` (size from the
 *     matching *_workspace_bytes function, 256-byte aligned).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls validate
 *     their arguments synchronously, enqueue their kernels on `stream` and
 *     return; results are ready once the stream has been synchronised.
 *   - Images are uint8, H rows of `pitch` bytes, pixel (y,x) channel c at
 *     img[y*pitch + x*C + c]; C in {1,2,3,4}; pitch >= W*C.
 *   - Energies are the e1 energy of the paper: sum over channels of
 *     |I(y,x+1)-I(y,x-1)| + |I(y+1,x)-I(y-1,x)| with indices clamped to the
 *     image (a border pixel takes a one-sided difference).
 *   - Seams are int32 column indices, one per row, top to bottom, in the
 *     coordinates of the image the seam was removed from.  Ties: the leftmost
 *     upper neighbour in the DP and the leftmost column of the last row, so the
 *     seam is unique (the minimum of the key (cost, s[H-1], ..., s[0])).
 *   - Limits: 1 <= H, W; H*510*C <= 8388000 (the cumulative cost of a column
 *     must fit 23 bits); W <= 65535.  Violations return SC_EUNSUPPORTED.
 *   - Errors are negative return codes; sc_last_error() gives the text.  No
 *     C++ exception crosses the ABI.  Device-side failures (a team barrier
 *     that timed out, a team not placed on one XCD) are reported through
 *     sc_read_status(): the image's results are then invalid.
 *   - Argument order: the arguments of the problem statement (image, its
 *     shape, the target, outputs, workspace, stream) come first; optional
 *     launch plumbing (a source image, a launch shape, extra outputs) trails,
 *     nullable.
 *   - Thread safety: calls are reentrant; calls that share a workspace must be
 *     ordered on one stream.
 */
#ifndef SEAMCARVE_SC_H
#define SEAMCARVE_SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sc_status;
enum {
    SC_OK = 0,
    SC_EINVAL = -1,      /* bad argument or shape */
    SC_ENOMEM = -2,      /* workspace too small */
    SC_EHIP = -3,        /* a HIP runtime call failed */
    SC_EBUSY = -4,       /* reserved for admission control */
    SC_EUNSUPPORTED = -5 /* outside the limits above */
};

/* Text of the last error on this thread (host memory, valid until the next sc_* call). */
const char* sc_last_error(void);

/* Library version string (host memory, static). */
const char* sc_version(void);

/*
 * Workspace bytes for sc_carve / sc_dp_seam on an image of H x W with C
 * channels (pure host function, no device access).  Returns 0 on bad args.
 */
size_t sc_workspace_bytes(int H, int W, int C);

/*
 * e1 energy map (sec. "Energy Mapping", first bullet of the paper).
 *   img    : H x W x C image, row pitch `pitch` bytes (read only).
 *   energy : H*W int32, dense row-major, written.
 */
sc_status sc_energy(const uint8_t* img, int H, int W, int C, int pitch, int32_t* energy, void* stream);

/*
 * Minimum vertical seam of a given energy map: the DP recurrence of the DP
 * section, the bottom-row argmin and the backtrack of Alg. 3.
 *   energy   : H*W int32, dense (read only).  Precondition: 0 <= e <= 65535
 *              and H*max(e) <= 8388000; otherwise the seam is unspecified
 *              (no fault).
 *   seam     : H int32, written.
 *   cost     : 1 int64, written (sum of e along the seam).
 *   ws       : workspace of at least sc_workspace_bytes(H, W, 1) bytes.
 * Trailing argument (nullable):
 *   dirs_out : H*W uint8 receives the parent direction of every cell
 *              (0 = upper-left, 1 = up, 2 = upper-right; row 0 is 1).
 */
sc_status sc_dp_seam(const int32_t* energy, int H, int W, int32_t* seam, int64_t* cost, void* ws, size_t ws_bytes,
                     void* stream, uint8_t* dirs_out);

/*
 * Remove one vertical seam (sec. "Removal of Seams"): in row i the pixels
 * right of column seam[i] move one column left; the width becomes W-1.  In
 * place at unchanged pitch; the bytes of the old last column stay as they were.
 *   seam : H int32, 0 <= seam[i] < W (device; out-of-range rows are skipped).
 */
sc_status sc_remove_seam(uint8_t* img, int H, int W, int C, int pitch, const int32_t* seam, void* stream);

/*
 * Transpose J(x,y,c) = I(y,x,c) (reduction of horizontal to vertical seams,
 * sec. "Design Techniques").  dst has W rows of dst_pitch >= H*C bytes.
 * src and dst must not overlap.
 */
sc_status sc_transpose_u8(const uint8_t* src, int H, int W, int C, int src_pitch, uint8_t* dst, int dst_pitch,
                          void* stream);

/* Launch shape of the persistent carve kernel; NULL selects the built-in choice. */
typedef struct {
    int team;    /* workgroups working together on one image (0 = default: 8 for sc_carve,
                    at most 16 per image in a batch; teams run on one XCD) */
    int variant; /* kernel variant id (see sc_variant_count); -1 = default */
    int flags;   /* SC_TUNE_* bits */
} sc_tune;

/* Remove every seam pixel by moving the pixels right of it (the paper's removal literally)
 * instead of moving whichever side of the row is shorter.  Results are identical. */
#define SC_TUNE_NO_MINSIDE 1
/* sc_carve (and the carve inside sc_insert_seams): bits 8..10 of flags name the XCD (0..7) the
 * team's workgroups run on, so that concurrent carves on different streams can use different
 * XCDs.  Default 0.  Results are identical. */
#define SC_TUNE_XCD_SHIFT 8
#define SC_TUNE_XCD(x) (((x) & 7) << SC_TUNE_XCD_SHIFT)

/* Number of compiled kernel variants and a description of variant v (host memory, static). */
int sc_variant_count(void);
const char* sc_variant_name(int v);

/*
 * Carve one image to target_w columns by removing W-target_w vertical seams
 * one at a time (the flowchart loop of the paper; each seam is the minimum
 * seam of the current image, Alg. 3 Require/Ensure: an n x m image in, an
 * n x m' image out).  One persistent kernel runs the whole loop on the device.
 *   img       : the image; on return the first target_w*C bytes of each row
 *               hold the result (pitch unchanged).
 *   target_w  : 1 <= target_w <= W; target_w == W copies src (if given) and
 *               removes nothing.
 *   pitch     : bytes per row of img (and of src), >= W*C.
 *   seams_out : nullable, (W-target_w)*H int32; seam k at seams_out[k*H + i].
 *   costs_out : nullable, (W-target_w) int64.
 *   ws        : workspace of at least sc_workspace_bytes(H, W, C) bytes.
 * Trailing arguments (both nullable):
 *   src       : the H x W x C source image (pitch `pitch`), read and written
 *               to img before carving (src is not modified); NULL carves img
 *               in place.
 *   tune      : host pointer to the launch shape; NULL = the built-in choice.
 * The arguments before `stream` are those of the problem statement in their
 * order; src and tune are launch plumbing and come last.
 */
sc_status sc_carve(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out, int64_t* costs_out,
                   void* ws, size_t ws_bytes, void* stream, const uint8_t* src, const sc_tune* tune);

/*
 * sc_carve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same carve, arguments and results as sc_carve, with its scratch in a fixed
 * array of SC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends, instead of a caller's workspace.  The call
 * allocates nothing (no hipMalloc, no library allocation).
 *   status_out : nullable device uint32, receives the device-side status of
 *                the carve (0 = fine, nonzero = the flags of sc_read_status:
 *                the results are then invalid).
 * Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * contents (the carve clears what must start at zero): calls that overlap on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller.  An image whose sc_workspace_bytes(H, W, C) exceeds
 * SC_NOALLOC_SCRATCH_BYTES (about 3840 x 2160 x 3 fits) returns SC_ENOMEM.
 */
#define SC_NOALLOC_SCRATCH_BYTES (64u << 20)
sc_status sc_carve_noalloc(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out,
                           int64_t* costs_out, uint32_t* status_out, void* stream, const uint8_t* src,
                           const sc_tune* tune);

/*
 * Seam insertion (the "Image Enlargement" subsection of the applications
 * section): widen img by k columns.  The k minimum seams are found by removal
 * on a copy, exactly as sc_carve(img -> W - k) removes them; img itself is not
 * modified.  Mapped to columns of the original image they are k distinct pixels
 * per row, and inserting the seams one by one in removal order places one new
 * pixel immediately right of each of them, whose value is the average of its
 * left and right neighbours, (a + b + 1) >> 1 per channel (a = the seam pixel,
 * b = the pixel to its right in img; a itself at the last column).
 *
 * img:       device, H rows of `pitch` bytes, W*C used (uint8, channels last).
 * out:       device, H rows of `out_pitch` bytes, (W + k)*C written; must not
 *            overlap img.
 * seams_out: nullable device int32 k*H: seam j's original column in row i at
 *            seams_out[j*H + i], in removal order.
 * tune:      launch shape of the carve that finds the seams (NULL = default).
 * ws:        device workspace of sc_insert_workspace_bytes(H, W, C, pitch, k)
 *            bytes, 256-byte aligned, owned by the caller.
 * Requires 0 <= k < W and W <= 65536.  Errors: SC_EINVAL (arguments),
 * SC_ENOMEM (workspace too small), SC_EUNSUPPORTED (W too large), SC_EHIP.
 * Asynchronous on `stream`.
 */
size_t sc_insert_workspace_bytes(int H, int W, int C, int pitch, int k);
sc_status sc_insert_seams(const uint8_t* img, int H, int W, int C, int pitch, int k, uint8_t* out, int out_pitch,
                          int32_t* seams_out, const sc_tune* tune, void* ws, size_t ws_bytes, void* stream);

/* One image of a batch (host struct; its pointers are device pointers). */
typedef struct {
    uint8_t* img;
    int H, W, C, pitch, target_w;
    int32_t* seams_out;  /* nullable */
    int64_t* costs_out;  /* nullable */
    const uint8_t* src;  /* nullable, as in sc_carve (launch plumbing, last) */
} sc_job;

/* Workspace bytes for a batch of n jobs (host array). 0 on bad args. */
size_t sc_batch_workspace_bytes(const sc_job* jobs, int n);

/* Summary of a prepared batch (host struct, filled by sc_batch_prepare). */
typedef struct {
    int n;        /* images */
    int nblocks;  /* workgroups of the carve launch */
    int variant;  /* kernel variant */
    int max_rows; /* tallest image */
    int team;       /* largest team of workgroups for one image */
    int teams_used; /* images carved by a team of more than one workgroup */
    size_t off_imgs, off_blk, off_teams, off_team_imgs; /* plan arrays inside ws */
} sc_batch_info;

/*
 * Batched carve, split in two so that the launch can be captured in a HIP
 * graph and replayed:
 *   sc_batch_prepare validates the jobs, plans which workgroups carve which
 *   image (images ordered by work, longest first; the workgroups of one team
 *   placed on one XCD) and writes the plan into ws with a synchronous copy;
 *   `info` (host) receives the summary that sc_batch_launch needs.
 *   sc_batch_launch enqueues the energy and carve kernels for that plan; it
 *   makes no host-to-device copy and allocates nothing.  Replaying it carves
 *   the jobs again from their src (jobs without src would be carved twice).
 *   tune: host pointer, nullable.
 */
sc_status sc_batch_prepare(const sc_job* jobs, int n, const sc_tune* tune, void* ws, size_t ws_bytes,
                           sc_batch_info* info);
sc_status sc_batch_launch(const sc_batch_info* info, void* ws, void* stream);

/* The two passes of sc_batch_launch, for callers that time them apart:
 * the energy pass (zero control words, copy src -> img, e1 energy of every image) and the
 * carve pass (the persistent kernel running the seam loop of every image). */
sc_status sc_batch_launch_energy(const sc_batch_info* info, void* ws, void* stream);
sc_status sc_batch_launch_carve(const sc_batch_info* info, void* ws, void* stream);

/* prepare + launch. */
sc_status sc_carve_batch(const sc_job* jobs, int n, const sc_tune* tune, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * Forward energy (sec. "Forward Energy Calculation": the cost of a seam is the
 * energy of the pixel pairs its removal makes neighbours).  The DP of Alg. 3
 * runs with the per-pixel energy replaced by those costs:
 *   CU(i,j) = D((i,j-1),(i,j+1)),
 *   M(i,j)  = min(M(i-1,j-1) + CU + D((i-1,j),(i,j-1)),
 *                 M(i-1,j)   + CU,
 *                 M(i-1,j+1) + CU + D((i-1,j),(i,j+1))),   M(0,j) = CU(0,j),
 * where D(p,q) is the sum over channels of |I(p)-I(q)| and a column index
 * outside the row is clamped to it (so a border pixel costs its difference to
 * the pixel that becomes the border).  Ties, backtrack, removal and the seam
 * loop are those of sc_carve; the costs are recomputed from the current pixels
 * for every seam.  A team of 256-thread workgroups on one XCD carves one
 * image: each DP member computes 976 columns and owns the middle 752; every
 * second 56-row phase the members exchange the keys of the 112 columns on
 * each side.  sc_carve_forward sizes the team so that every wave walks and
 * removes about 8 rows of a seam (at most 32 workgroups).
 *
 * sc_carve_forward: arguments as sc_carve (no tune); seams_out/costs_out
 *   (nullable) receive every seam and its forward cost.  ws: at least
 *   sc_forward_workspace_bytes(H, W, C) bytes, 256-byte aligned.
 * Batches: sc_forward_batch_prepare validates the jobs and writes the image
 *   descriptors into ws with a synchronous copy (ws: at least
 *   sc_forward_batch_workspace_bytes(jobs, n) bytes); sc_forward_batch_launch
 *   enqueues the copy-in pass and the carve (no allocation, no host copy; the
 *   info must come from sc_forward_batch_prepare).  Per-image clocks:
 *   sc_read_times on the same ws.
 * Limits: those of sc_carve, plus W <= 8192 and H*roundup(W*C, 64) < 2^31.
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_EUNSUPPORTED, SC_EHIP.
 */
size_t sc_forward_workspace_bytes(int H, int W, int C);
sc_status sc_carve_forward(uint8_t* img, int H, int W, int C, int target_w, int pitch, int32_t* seams_out,
                           int64_t* costs_out, void* ws, size_t ws_bytes, void* stream, const uint8_t* src);
size_t sc_forward_batch_workspace_bytes(const sc_job* jobs, int n);
sc_status sc_forward_batch_prepare(const sc_job* jobs, int n, void* ws, size_t ws_bytes, sc_batch_info* info);
sc_status sc_forward_batch_launch(const sc_batch_info* info, void* ws, void* stream);
/* The two passes of sc_forward_batch_launch, for callers that time them apart: the copy-in pass
 * (zero control words, copy src -> img and into the working copy) and the carve. */
sc_status sc_forward_batch_launch_copy(const sc_batch_info* info, void* ws, void* stream);
sc_status sc_forward_batch_launch_carve(const sc_batch_info* info, void* ws, void* stream);

/*
 * Object removal with a mask (the "Object Removal" subsection of the
 * applications section): the pixels of a binary mask get a very large
 * negative energy, so the minimum seam runs through the object while any of it
 * is left, and seams are removed from the image and from the mask alike until
 * no masked pixel remains; optionally as many seams are then inserted to
 * restore the size.  Precisely:
 *   - masked energy: the e1 energy of the current image minus
 *     B = h*510*C + 1 at every masked pixel (h = rows of the carved frame).  B
 *     exceeds the e1 energy of any seam, so the minimum seam has the most
 *     masked pixels, then the least energy, then the leftmost ties of sc_carve;
 *   - direction: direction = SC_OBJ_AUTO takes the mask's bounding box, h_m
 *     rows by w_m columns: vertical seams when w_m <= h_m (or the mask is
 *     empty), horizontal seams (carved on the transpose) otherwise;
 *   - loop: while a masked pixel is left and the frame has more than one
 *     column, remove the minimum masked seam from the image and the mask;
 *   - restore (restore = 1): the k removed columns come back by seam insertion
 *     (sc_insert_seams) on the reduced frame, in rounds of at most
 *     (current width - 1) seams; a reduced frame of one column gives SC_EINVAL.
 * Arguments:
 *   img, mask : H x W x C image (pitch bytes per row) and H x W mask (mpitch
 *               bytes per row; any nonzero byte marks a pixel); not modified.
 *   direction : SC_OBJ_AUTO, SC_OBJ_VERTICAL or SC_OBJ_HORIZONTAL.
 *   out       : result, out_pitch >= W*C bytes per row, H rows available,
 *               must not overlap img or mask: info->rows x info->cols pixels
 *               (H x W when restoring; H x (W-k) for vertical seams,
 *               (H-k) x W for horizontal ones otherwise).
 *   info      : host struct, filled on success.
 *   seams_out : nullable, H*W int32: seam j at seams_out[j*h + i], i < h, in
 *               the frame that was carved (h = H vertical, W horizontal) and
 *               the columns of the frame it was removed from.
 *   costs_out : nullable, max(H, W) int64: the masked cost of every seam
 *               (sum of e1 minus B times its masked pixels).
 *   ws        : at least sc_object_workspace_bytes(H, W, C, restore) bytes,
 *               256-byte aligned.
 * Synchronous: the frame and the output size depend on the mask, so the call
 * waits for the device (after the mask extent and after the carve) and
 * returns with out complete.  One 1024-thread workgroup carves the frame.
 * Limits: carved frame of at most 8192 columns and rows*510*C <= 8388000.
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_EUNSUPPORTED, SC_EHIP.
 */
#define SC_OBJ_AUTO (-1)
#define SC_OBJ_VERTICAL 0
#define SC_OBJ_HORIZONTAL 1
typedef struct {
    int32_t direction; /* the direction used */
    int32_t k;         /* seams removed (and inserted back when restoring) */
    int32_t rows, cols; /* size of out */
    int32_t left;      /* masked pixels left (0 unless the frame reached one column first) */
    int32_t pad;
    double carve_ms;    /* device time of the masked carve */
    double stage_ms[3]; /* of which: DP sweep; argmin and backtrack; removal */
} sc_object_info;
size_t sc_object_workspace_bytes(int H, int W, int C, int restore);
sc_status sc_remove_object(const uint8_t* img, const uint8_t* mask, int H, int W, int C, int pitch, int mpitch,
                           int direction, int restore, uint8_t* out, int out_pitch, sc_object_info* info,
                           int32_t* seams_out, int64_t* costs_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Step-wise carving for a serving loop (continuous batching).  A slot table (device memory,
 * sc_slot_table_bytes(n) bytes, caller-owned) holds one image per slot; each image keeps its own
 * workspace (sc_workspace_bytes) and stays on the device between steps.
 *   sc_slot_start  validates the job and 0 <= slot < n_slots (the table's size as passed to
 *                  sc_slot_table_bytes), writes the job's descriptor into slot `slot` and
 *                  enqueues its energy pass (copying job->src into job->img when src is given).
 *   sc_slot_clear  empties slot `slot` (0 <= slot < n_slots; its workspace may then be reused).
 *   sc_slots_step  advances every non-empty slot of the first n by at most max_seams seams in one
 *                  launch (one workgroup per image) and writes progress[i] = seams removed so far
 *                  (device int32; -1 = device error, -2 = empty slot).  A slot is done when
 *                  progress equals W - target_w.  Calls that share a table must be ordered on
 *                  one stream.
 *   sc_slots_step_timed  the same with a time budget: each image's workgroup stops after the
 *                  first seam that ends budget_us microseconds (device wall clock) or more after
 *                  it started in this launch, or after max_seams seams; budget_us = 0 is
 *                  sc_slots_step.  A step's workgroups then stay busy for about the same time
 *                  instead of waiting for the one with the most work.
 *   sc_slots_step_teams  sc_slots_step_timed where slot s is carved by a team of team[s]
 *                  workgroups (host array of n_slots entries, 1 = one workgroup, at most 32);
 *                  table_slots is the table's size as passed to sc_slot_table_bytes (>= n_slots):
 *                  the teams sit on one XCD each and are resident together (a team that finds
 *                  no room in this step carves with one workgroup); the budget is the team's
 *                  first member's.  Results equal those of sc_slots_step_timed.  The call writes
 *                  the step's block plan into the table (after the descriptors) with an
 *                  asynchronous host-to-device copy from pageable memory.
 */
size_t sc_slot_table_bytes(int n_slots);
sc_status sc_slot_start(const sc_job* job, void* ws, size_t ws_bytes, void* table, int n_slots, int slot,
                        void* stream);
sc_status sc_slot_clear(void* table, int n_slots, int slot, void* stream);
sc_status sc_slots_step(const void* table, int n_slots, int max_seams, int32_t* progress, void* stream);
sc_status sc_slots_step_timed(const void* table, int n_slots, int max_seams, long long budget_us, int32_t* progress,
                              void* stream);
sc_status sc_slots_step_teams(const void* table, int table_slots, int n_slots, const int32_t* team, int max_seams,
                              long long budget_us, int32_t* progress, void* stream);

/*
 * Device-side status of the images of a workspace (synchronous: waits for the
 * device).  flags[i] for image i (n = 1 for sc_carve/sc_dp_seam workspaces):
 * 0 = fine, bit 0 = a team barrier timed out (the results of that image are
 * invalid).  Returns the number of images written.
 */
int sc_read_status(const void* ws, uint32_t* flags, int max_n);

/*
 * Device clock stamps of the images of a workspace (synchronous): t_begin[i] / t_end[i] are
 * the constant-rate device clock (s_memrealtime) when the carve of image i started and ended;
 * *hz receives that clock's rate.  Returns the number of images written, -1 on error.
 */
int sc_read_times(const void* ws, uint64_t* t_begin, uint64_t* t_end, int max_n, double* hz);

/*
 * Device clock ticks (rate as in sc_read_times) each image's carve spent in its three stages,
 * summed over its seams, as seen by its first workgroup (synchronous): stages[3*i + 0] the DP
 * sweep with the bottom-row argmin, [3*i + 1] the backtrack and the removal, [3*i + 2] the band
 * energy update.  Returns the number of images written, -1 on error.
 */
int sc_read_stages(const void* ws, uint64_t* stages, int max_n);

#ifdef __cplusplus
}
#endif
#endif /* SEAMCARVE_SC_H */
