// HIP kernels of the seam-carving hot path for gfx950 (CDNA4).
//
// Steps (arXiv 2410.21207): e1 energy (sec. "Energy Mapping"), the DP table
// M(i,j) = e(i,j) + min(M(i-1,j-1..j+1)) (DP section, Alg. 3), the bottom-row
// argmin, the backtrack (Alg. 3) and the removal of the seam (sec. "Removal of
// Seams"), repeated once per seam on the current image (flowchart loop).
//
// Design (nothing here is a contraction, so no MFMA; every step is integer):
//  * The energy plane is kept on the device as uint16 (max e = 510*C <= 2040).
//  * The DP keeps a row of packed 32-bit keys in registers: bits [31:9] hold
//    M, bits [8:2] an ancestor offset, bits [1:0] the direction tag.  Each lane
//    owns CPL consecutive columns; neighbours in other lanes arrive through DPP
//    wave shifts.  The three parent candidates get tags 0/1/2 (left, up,
//    right) so one v_min3 picks the minimum AND the leftmost tie (reading R5),
//    and the same add moves the ancestor offset.  The direction bits are
//    shifted into a byte per lane with v_alignbit (half a byte with CPL 2,
//    which a lane pair joins) and stored as a 2-bit map.
//  * A wave owns a strip of S = 64*CPL - 2*KR columns and computes KR halo
//    columns on each side, so it runs KR rows with no exchange at all
//    ("ghost zone" tiling); waves exchange the last row of every KR-row phase
//    through memory and a barrier.
//  * At the last row of each phase every owned column records how far its
//    minimal path moved within the phase; the backtrack then hops phase by
//    phase (one load per phase) and walks the KR rows of every phase in
//    parallel from an LDS window of the direction map.
//  * Removal shifts the shorter side of each row one pixel toward the seam
//    (the right side only when min-side removal is off), row-parallel with
//    coalesced 16-byte slots, for the image and the energy plane alike;
//    the energy is then recomputed only at the two new columns {s-1, s} of
//    each row (the only cells whose stencil changed).
#include <mutex>

#include "sc_device.h"

namespace sc {

constexpr uint32_t QINF = 0xFFFFFF00u;  // "+infinity" key: larger than any real key, +10 cannot wrap

// r + 512 * (low or high 16 bits of `pair`): one v_mad_u32_u16 adds e(i,j) << 9 to a DP key
// straight from the packed uint16 energy pair, with no separate unpack.
__device__ __forceinline__ uint32_t mad_lo16(uint32_t pair, uint32_t r) {
    uint32_t o;
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(o) : "v"(pair), "s"(512u), "v"(r));
    return o;
}
__device__ __forceinline__ uint32_t mad_hi16(uint32_t pair, uint32_t r) {
    uint32_t o;
    asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(o) : "v"(pair), "s"(512u), "v"(r));
    return o;
}

// ----------------------------------------------------------------------------------------------
// e1 energy at one pixel of the current image (width w), indices clamped to the image.
template <bool COH = false>
__device__ __forceinline__ uint32_t energy_at(const uint8_t* img, long long pitch, int H, int w, int C, int y,
                                              int x) {
    const int xl = x > 0 ? x - 1 : 0, xr = x + 1 < w ? x + 1 : w - 1;
    const int yu = y > 0 ? y - 1 : 0, yd = y + 1 < H ? y + 1 : H - 1;
    const uint8_t* r = img + (long long)y * pitch;
    const uint8_t* ru = img + (long long)yu * pitch;
    const uint8_t* rd = img + (long long)yd * pitch;
    uint32_t s = 0;
    for (int c = 0; c < C; ++c) {
        const int dx = (int)ld<COH>(r + xr * C + c) - (int)ld<COH>(r + xl * C + c);
        const int dy = (int)ld<COH>(rd + x * C + c) - (int)ld<COH>(ru + x * C + c);
        s += (uint32_t)(dx < 0 ? -dx : dx) + (uint32_t)(dy < 0 ? -dy : dy);
    }
    return s;
}

// e1 energy at logical column x of a row from a buffer: the row starts at byte offset br of the
// descriptor's memory, the rows above and below at bu and bd (min-side removal keeps every row at
// its own offset).  The channel loop runs to 4 with dropped offsets past C, so the loads carry no
// branches and go out together; a column outside [0, w) is clamped like the pixels of any other
// (callers do not store its value).
template <bool COH>
__device__ __forceinline__ uint32_t energy_buf(__amdgpu_buffer_rsrc_t rb, uint32_t br, uint32_t bu, uint32_t bd, int w,
                                               int C, int x) {
    x = min(max(x, 0), w - 1);
    const int xl = x > 0 ? x - 1 : 0, xr = x + 1 < w ? x + 1 : w - 1;
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool ok = c < C;
        const int a = (int)buf_ld8<COH>(rb, ok ? br + (uint32_t)(xr * C + c) : kBufDrop);
        const int b = (int)buf_ld8<COH>(rb, ok ? br + (uint32_t)(xl * C + c) : kBufDrop);
        const int dn = (int)buf_ld8<COH>(rb, ok ? bd + (uint32_t)(x * C + c) : kBufDrop);
        const int up = (int)buf_ld8<COH>(rb, ok ? bu + (uint32_t)(x * C + c) : kBufDrop);
        s += (uint32_t)abs(a - b) + (uint32_t)abs(dn - up);
    }
    return s;
}

// Standalone energy map (int32, dense).
__global__ void energy_i32_kernel(const uint8_t* __restrict__ img, int H, int W, int C, long long pitch,
                                  int32_t* __restrict__ out) {
    const int y = blockIdx.y;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < W; x += gridDim.x * blockDim.x)
        *gp(out + (long long)y * W + x) = (int32_t)energy_at(img, pitch, H, W, C, y, x);
}


// A single-image workspace starts with a header: magic, image count, then the descriptor itself
// (read by the step-wise carve kernel), then the image's Ctl block.
__device__ __forceinline__ void write_single_header(const Img& d) {
    char* h = reinterpret_cast<char*>(d.amin) - kWsHeadBytes;
    reinterpret_cast<uint32_t*>(h)[0] = kWsMagic;
    reinterpret_cast<uint32_t*>(h)[1] = 1u;
    *reinterpret_cast<Img*>(h + kWsImgOffset) = d;
}

// Per-image preparation: reset the control words, optionally copy src -> img, fill the energy plane.
// Zero both DP exchange rows: a published key carries its phase's tag (never 0), so nothing a
// previous launch left there can pass for a key of this one.
__device__ __forceinline__ void clear_exchange(const Img& d) {
    for (int x = threadIdx.x; x < 2 * d.xw; x += blockDim.x) *gp(d.xq + x) = 0u;
}

// The energy pass (a1) and the copy into the working image.  The carve works on the copy in wk;
// img receives the result at the end (a carve that removes nothing copies src into img here).
//
// A workgroup sweeps one tile: a strip of 1024 columns (4 per thread) down kTileRows rows.  Each
// source row is read once per tile, as the aligned dwords covering the thread's 4 pixels and one
// pixel on each side, realigned to the row start with v_alignbyte (rows may start anywhere); the
// rows above and below stay in registers as the tile moves down.  The energy goes out as one
// 8-byte store of 4 uint16 per thread, the pixels as C dword stores into the 64-byte aligned rows
// of wk.
constexpr int kTileRows = 32;
constexpr int kTileCols = 1024;  // 256 threads x 4 pixels

template <int C>
__device__ void prepare_tile(const Img& d, const uint8_t* srcimg, int y0, int y1, int xs) {
    const int t = threadIdx.x, x0 = xs + 4 * t, H = d.H, W = d.W;
    const bool act = x0 < W;
    const bool identity = d.src && d.target_w == d.W;
    SrcRow<C> up, cur, dn;
    up.load(srcimg, d.pitch, W, max(y0 - 1, 0), x0);
    cur.load(srcimg, d.pitch, W, y0, x0);
    dn.load(srcimg, d.pitch, W, min(y0 + 1, H - 1), x0);
#pragma unroll 1
    for (int y = y0; y < y1; ++y) {
        SrcRow<C> nx;
        if (y + 1 < y1) nx.load(srcimg, d.pitch, W, min(y + 2, H - 1), x0);
        if (act) {
            if (d.e) {
                uint32_t e[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int x = x0 + p;
                    const uint32_t l = x > 0 ? cur.px(p - 1) : cur.px(p);
                    const uint32_t rr = x + 1 < W ? cur.px(p + 1) : cur.px(p);
                    e[p] = __builtin_amdgcn_sad_u8(up.px(p), dn.px(p), __builtin_amdgcn_sad_u8(l, rr, 0u));
                }
                uint16_t* er = d.e + (long long)y * d.ep + x0;
                if (x0 + 3 < W) {
                    *gp(reinterpret_cast<v2u*>(er)) = v2u{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
                } else {
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        if (x0 + p < W) *gp(er + p) = (uint16_t)e[p];
                }
            }
            uint32_t* wr = reinterpret_cast<uint32_t*>(d.wk + (long long)y * d.wp + (long long)x0 * C);
#pragma unroll
            for (int m = 0; m < C; ++m)
                if (x0 * C + 4 * m < W * C) *gp(wr + m) = cur.r[m + 1];
            if (identity) {
                uint8_t* o = d.img + (long long)y * d.pitch + (long long)x0 * C;
#pragma unroll
                for (int b = 0; b < 4 * C; ++b)
                    if (x0 * C + b < W * C) *gp(o + b) = (uint8_t)(cur.r[1 + (b >> 2)] >> (8 * (b & 3)));
            }
        }
        up = cur;
        cur = dn;
        dn = nx;
    }
}

// Tiles tile0, tile0 + tstep, ... of one image (tiles numbered strip-major within row chunks);
// tile 0 also resets the control words and clears the exchange rows.
__device__ void prepare_image(const Img& d, int tile0, int tstep) {
    const uint8_t* srcimg = d.src ? d.src : d.img;
    if (tile0 == 0) {
        if (threadIdx.x == 0) reset_ctl(d);
        clear_exchange(d);
    }
    const int ns = (d.W + kTileCols - 1) / kTileCols, nc = (d.H + kTileRows - 1) / kTileRows;
    for (int tile = tile0; tile < ns * nc; tile += tstep) {
        const int strip = tile % ns, chunk = tile / ns;
        const int y0 = chunk * kTileRows, y1 = min(d.H, y0 + kTileRows);
        if (strip == 0 && (int)threadIdx.x < y1 - y0) *gp(d.ro + y0 + threadIdx.x) = 0;
        switch (d.C) {
            case 1: prepare_tile<1>(d, srcimg, y0, y1, strip * kTileCols); break;
            case 2: prepare_tile<2>(d, srcimg, y0, y1, strip * kTileCols); break;
            case 3: prepare_tile<3>(d, srcimg, y0, y1, strip * kTileCols); break;
            default: prepare_tile<4>(d, srcimg, y0, y1, strip * kTileCols); break;
        }
    }
}

__global__ __launch_bounds__(256) void prepare_single_kernel(Img d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) write_single_header(d);
    prepare_image(d, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void prepare_batch_kernel(const Img* __restrict__ imgs, int n) {
    const int i = blockIdx.y;
    if (i < n) {
        const Img d = imgs[i];
        prepare_image(d, blockIdx.x, gridDim.x);
    }
}

// Energy plane from a caller's int32 energy map (sc_dp_seam).
__global__ void prepare_from_i32_kernel(Img d, const int32_t* __restrict__ e) {
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        if (threadIdx.x == 0) {
            write_single_header(d);
            reset_ctl(d);
        }
        clear_exchange(d);
    }
    const int y = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x == 0) *gp(d.ro + y) = 0;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < d.W; x += gridDim.x * blockDim.x)
        *gp(d.e + (long long)y * d.ep + x) = (uint16_t)*gp(e + (long long)y * d.W + x);
}

// ----------------------------------------------------------------------------------------------
// In-place left shift of row segments by one pixel, one wave.  Segment a: dst bytes [a_lo, a_hi)
// get src bytes shifted by sh_a (1..4); segment b likewise (sh_b).  The work is cut into 16-byte
// slots aligned to absolute addresses; a pass gives each lane U slots of the concatenated slot
// list and issues every load of the pass before any store.  A slot's store writes only inside the
// slot, and the bytes it needs beyond its end belong to the next slot of the same segment, which
// is loaded in the same pass or a later one -- so the in-place update is hazard free.
struct Seg {
    uint8_t* base;  // 16-byte aligned (wave-uniform)
    int lo, hi;     // the segment is [base + lo, base + hi)
    int sh;         // shift in bytes, 1..4
    int n;          // 16-byte slots covering it
};

__device__ __forceinline__ Seg make_seg(uint8_t* lo_p, uint8_t* hi_p, int sh) {
    Seg g;
    const int off = (int)((uintptr_t)lo_p & 15);
    g.base = lo_p - off;
    g.lo = off;
    g.hi = hi_p > lo_p ? off + (int)(hi_p - lo_p) : off;
    g.sh = sh;
    g.n = g.hi > g.lo ? ((g.hi - 1) >> 4) + 1 : 0;
    return g;
}

template <int U, bool COH>
__device__ __forceinline__ void seg_load(const Seg& g, int fb, int lane, uint32_t (&D)[U][5]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = fb + u * 64 + lane;
#pragma unroll
        for (int i = 0; i < 5; ++i) D[u][i] = 0;
        if (f < g.n) {
            const uint32_t so = (uint32_t)f << 4;  // slot offset from the uniform base
            const uint64_t* q = reinterpret_cast<const uint64_t*>(g.base + so);
            const uint64_t v0 = ld<COH>(q), v1 = ld<COH>(q + 1);
            D[u][0] = (uint32_t)v0; D[u][1] = (uint32_t)(v0 >> 32);
            D[u][2] = (uint32_t)v1; D[u][3] = (uint32_t)(v1 >> 32);
            if ((int)so + 16 - g.sh < g.hi) D[u][4] = ld<COH>(reinterpret_cast<const uint32_t*>(g.base + so + 16));
        }
    }
}

template <int U>
__device__ __forceinline__ void seg_store(const Seg& g, int fb, int lane, const uint32_t (&D)[U][5]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = fb + u * 64 + lane;
        if (f >= g.n) continue;
        const int so = f << 4;
        uint8_t* sp = g.base + so;
        uint32_t o[4];
        if (g.sh == 4) {
            o[0] = D[u][1]; o[1] = D[u][2]; o[2] = D[u][3]; o[3] = D[u][4];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbyte(D[u][i + 1], D[u][i], (uint32_t)g.sh);
        }
        if (so >= g.lo && so + 16 <= g.hi) {
            *gp(reinterpret_cast<u32x4*>(sp)) = u32x4{o[0], o[1], o[2], o[3]};
        } else {
            // a slot at a segment edge: store only the bytes inside the segment, one predicated
            // byte store per position (static offsets and register indices)
            const int k0 = so > g.lo ? 0 : g.lo - so;
            const int k1 = so + 16 < g.hi ? 16 : g.hi - so;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k >= k0 && k < k1) *gp(sp + k) = (uint8_t)(o[k >> 2] >> ((k & 3) * 8));
        }
    }
}

// In-place left shift of up to two row segments by one pixel, one wave.  Segment a: the bytes
// of [a_lo, a_hi) take the values sh_a bytes to their right; segment b likewise.  The work is
// cut into 16-byte slots aligned to absolute addresses; a pass gives each lane U slots of each
// segment and issues every load of the pass before any store.  A slot's store writes only inside
// the slot, and the bytes it needs beyond its end belong to the next slot of the same segment,
// loaded in the same pass or a later one -- so the in-place update is hazard free.
template <int U, bool COH>
__device__ __forceinline__ void shift_segments_wave(uint8_t* a_lo_p, uint8_t* a_hi_p, int sh_a, uint8_t* b_lo_p,
                                                    uint8_t* b_hi_p, int sh_b, int lane) {
    const Seg A = make_seg(a_lo_p, a_hi_p, sh_a);
    const Seg B = make_seg(b_lo_p, b_hi_p, sh_b);
    const int n = max(A.n, B.n);
#pragma unroll 1
    for (int fb = 0; fb < n; fb += 64 * U) {
        uint32_t DA[U][5], DB[U][5];
        seg_load<U, COH>(A, fb, lane, DA);
        seg_load<U, COH>(B, fb, lane, DB);
        seg_store<U>(A, fb, lane, DA);
        seg_store<U>(B, fb, lane, DB);
    }
}

// Standalone seam removal: one wave per row.
__global__ void remove_seam_kernel(uint8_t* __restrict__ img, int H, int W, int C, long long pitch,
                                   const int32_t* __restrict__ seam) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int y = wv; y < H; y += nw) {
        const int s = *gp(seam + y);
        if (s < 0 || s >= W) continue;
        uint8_t* row = img + (long long)y * pitch;
        shift_segments_wave<4, false>(row + (long long)s * C, row + (long long)(W - 1) * C, C, row, row, 1, lane);
    }
}

// ----------------------------------------------------------------------------------------------
// Transpose J(x,y,c) = I(y,x,c) through a 64x64-pixel LDS tile.
template <int C>
__global__ void transpose_kernel(const uint8_t* __restrict__ src, int H, int W, long long sp,
                                 uint8_t* __restrict__ dst, long long dp) {
    __shared__ uint8_t tile[64][64 * C + 4];
    const int bx = blockIdx.x * 64, by = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 256 threads: 4 rows per pass
    for (int r = ty; r < 64; r += 4) {
        const int y = by + r, x = bx + tx;
        if (y < H && x < W)
            for (int c = 0; c < C; ++c) tile[r][tx * C + c] = *gp(src + (long long)y * sp + (long long)x * C + c);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int x = bx + r, y = by + tx;  // output row x, column y
        if (y < H && x < W)
            for (int c = 0; c < C; ++c) *gp(dst + (long long)x * dp + (long long)y * C + c) = tile[tx][r * C + c];
    }
}

// ----------------------------------------------------------------------------------------------
// The carve engine: one image, carved by a team of G workgroups of NT threads.
template <int CPL, int KR, int NT>
struct Carver {
    static constexpr int WIN = 64 * CPL;       // columns a wave computes
    static constexpr int S = WIN - 2 * KR;     // columns a wave owns
    static constexpr int NW = NT / 64;         // waves per workgroup
    static constexpr int PF = 8;                         // rows of energy prefetched ahead
    static constexpr int WD = (KR / 2 + 2 + 3) / 4 + 1;  // dwords of a backtrack window row
    static constexpr int PMAX = 16448 / KR + 2;          // phases of the tallest image
    static_assert(CPL == 2 || CPL == 4 || CPL == 8, "a lane's directions fill half a byte, a byte or a short");
    static_assert(KR % CPL == 0 && KR % PF == 0 && KR <= 63 && S > 0 && S % 16 == 0, "phase shape");

    struct Smem {
        uint32_t xs[2][kLdsExchangeMaxW];  // phase exchange rows of a single-workgroup carve
        int jend[PMAX];                    // seam column at the last row of every phase
        uint32_t win[NW][KR * WD];         // backtrack windows of the direction map
        int chain;                         // jend[p] is final for every p >= chain
        int flag;
        int stop;                          // step mode: the time budget is spent
    };

    struct EV {
        uint64_t v[(CPL + 3) / 4];  // CPL uint16 energies
    };

    // Energies at the lane's byte offset `off` (a valid column) of the row starting `soff` bytes
    // into the plane (wave-uniform: row base plus the row's start offset): a buffer load with the
    // row part in a scalar register.  COH sets the sc1 bit.
    template <bool COH>
    static __device__ __forceinline__ EV load_ev(__amdgpu_buffer_rsrc_t re, uint32_t soff, uint32_t off) {
        EV e;
        if constexpr (CPL == 2) {
            e.v[0] = __builtin_amdgcn_raw_buffer_load_b32(re, (int)off, (int)soff, COH ? 16 : 0);
        } else if constexpr (CPL == 4) {
            const v2u v = __builtin_amdgcn_raw_buffer_load_b64(re, (int)off, (int)soff, COH ? 16 : 0);
            e.v[0] = ((uint64_t)v[1] << 32) | v[0];
        } else {
            const v4u v = __builtin_amdgcn_raw_buffer_load_b128(re, (int)off, (int)soff, COH ? 16 : 0);
            e.v[0] = ((uint64_t)v[1] << 32) | v[0];
            e.v[1] = ((uint64_t)v[3] << 32) | v[2];
        }
        return e;
    }

    // One DP row for the CPL columns of this lane.  Q holds the previous row's keys (the tag bits
    // [1:0] are ignored); on return Q holds this row's keys and the result's top 2*CPL bits hold
    // this row's directions, column 0 lowest.  EDGE: the window reaches past the image; a column
    // outside [0, w) must never be a parent, so the candidates that cross the image's edges are
    // made all ones by saturating adds of per-lane words (radd[j]: 10, or all ones when column j
    // is outside; ladd: 0, or all ones when the lane's last column is outside).  The keys of the
    // outside columns themselves are never read.
    template <bool EDGE>
    static __device__ __forceinline__ uint32_t row_step(uint32_t (&Q)[CPL], const EV& ev, const uint32_t (&radd)[CPL],
                                                        uint32_t ladd) {
        uint32_t t[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) t[k] = Q[k] & ~3u;
        // The neighbours of the lane's first and last column live in lanes -1 and +1.  At the
        // wave's edges the shift fills in 0: those columns are halo, and within a phase a wrong
        // value there moves at most one column inward per row, never reaching an owned column.
        const uint32_t left = (uint32_t)__builtin_amdgcn_update_dpp(
            0, (int)(EDGE ? __builtin_elementwise_add_sat(t[CPL - 1], ladd) : t[CPL - 1]), 0x138, 0xf, 0xf, true);
        const uint32_t rightR = (uint32_t)__builtin_amdgcn_update_dpp(
            0, (int)(EDGE ? __builtin_elementwise_add_sat(t[0], radd[0]) : t[0] + 10u), 0x130, 0xf, 0xf, true);
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const uint32_t L = k ? t[k - 1] : left;                      // tag 0, offset +0
            const uint32_t Cc = t[k] + 5u;                               // tag 1, offset +1
            const uint32_t R = k + 1 < CPL ? (EDGE ? __builtin_elementwise_add_sat(t[k + 1], radd[k + 1]) : t[k + 1] + 10u)
                                           : rightR;                     // tag 2, offset +2
            const uint32_t r = min(min(L, Cc), R);
            const uint32_t pair = (uint32_t)(ev.v[k >> 2] >> (((k >> 1) & 1) * 32));
            Q[k] = (k & 1) ? mad_hi16(pair, r) : mad_lo16(pair, r);
            acc = __builtin_amdgcn_alignbit(r, acc, 2u);
        }
        return acc;
    }

    struct Next {
        bool valid, lane_any;
        int r0, r1;
        uint32_t off;  // byte offset of the lane's first column in an energy row
    };

    static __device__ __forceinline__ Next make_next(const Img& d, int w, int p, int t, int lane, bool valid) {
        Next nx;
        nx.valid = valid;
        nx.r0 = __builtin_amdgcn_readfirstlane(p * KR);  // wave-uniform: a scalar buffer offset
        nx.r1 = min(d.H, nx.r0 + KR);
        const int col0 = t * S - KR + lane * CPL;
        nx.lane_any = valid && col0 >= 0 && col0 < w;
        nx.off = (uint32_t)(nx.lane_any ? col0 : 0) * 2u;
        return nx;
    }

    // One strip (t) of one phase (p) for the calling wave.  `ring` holds the first PF rows when
    // `preloaded`; when this phase's length is a multiple of PF, its last block of rows prefetches
    // the first PF rows of the wave's next item `nx`, so the energy stream runs across phase
    // boundaries.  The row loop has no lane-dependent branches: every load targets a valid row and
    // column, and lanes that do not own their columns store their directions to a dropped offset.
    // Tag of the keys published at global phase g (seam k, phase p: g = k * P + p): 1..511, never
    // the 0 of a cleared exchange row.  Two phases apart the tags differ, which is all a reader
    // of the double-buffered rows needs.
    static __device__ __forceinline__ uint32_t phase_tag(int g) { return 1u + (uint32_t)g % 511u; }

    // Returns false when the wait for a neighbour's keys timed out (the image's status says so).
    template <bool EDGE, bool TEAM>
    // `rovc` carries the row start offsets of the next item (lane l: its row l) from one item to
    // the next together with the prefetched energy rows.
    static __device__ __forceinline__ bool dp_item(const Img& d, Smem& sm, int w, int p, int t, int lane,
                                                   EV (&ring)[PF], bool preloaded, const Next& nx, int gk,
                                                   int& rovc) {
        const int r0 = __builtin_amdgcn_readfirstlane(p * KR), r1 = min(d.H, r0 + KR);
        const int base = t * S - KR;
        const int col0 = base + lane * CPL;
        const bool lane_any = col0 >= 0 && col0 < w;
        const bool owned = lane >= KR / CPL && lane < (KR + S) / CPL && col0 < w;
        bool valid[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) valid[k] = (col0 + k >= 0) && (col0 + k < w);

        const uint32_t eoff = (uint32_t)(lane_any ? col0 : 0) * 2u;  // lanes off the image read column 0
        const uint32_t erb = (uint32_t)d.ep * 2u;                       // bytes per energy row
        const __amdgpu_buffer_rsrc_t re = make_rsrc(d.e, (uint32_t)d.H * erb);
        const __amdgpu_buffer_rsrc_t rdir = make_rsrc(d.dirs, (uint32_t)((d.H + 3) & ~3) * (uint32_t)d.db);
        // start offsets of this item's rows and of the next item's rows: lane l holds row r0 + l.
        // A preloaded item got its own from the previous item, so its first prefetch does not wait.
        const int last = d.H - 1;
        const __amdgpu_buffer_rsrc_t rro = make_rsrc(d.ro, (uint32_t)d.H * 4u);
        const int rov = preloaded ? rovc : (int)buf_ld32<TEAM>(rro, lane < KR ? (uint32_t)min(r0 + lane, last) * 4u : kBufDrop);
        const int rovn = (int)buf_ld32<TEAM>(rro, lane < KR ? (uint32_t)min(nx.r0 + lane, last) * 4u : kBufDrop);
        rovc = rovn;
        // byte offset in the energy plane of row r0 + l (row base plus the row's start offset) in
        // lane l, rows past the image clamped to the last one; a row's scalar buffer offset is
        // then one readlane
        const uint32_t roff = (uint32_t)min(r0 + lane, last) * erb + 2u * (uint32_t)rov;
        const uint32_t roffn = (uint32_t)min(nx.r0 + lane, last) * erb + 2u * (uint32_t)rovn;
        auto soff = [&](int i) { return (uint32_t)__builtin_amdgcn_readlane(roff, i); };    // i < KR
        auto soffn = [&](int i) { return (uint32_t)__builtin_amdgcn_readlane(roffn, i); };  // i < PF
        if (!preloaded) {
#pragma unroll
            for (int i = 0; i < PF; ++i) ring[i] = load_ev<TEAM>(re, soff(i), eoff);
        }
        // previous row's keys.  Phase 0 starts from a row of zeros: one ordinary DP step then gives
        // M(0,j) = e(0,j) (its directions and offsets are never read).
        uint32_t Q[CPL];
        if (p == 0) {
#pragma unroll
            for (int k = 0; k < CPL; ++k) Q[k] = valid[k] ? 0u : QINF;
        } else {
            const int cx = lane_any ? col0 : 0;
            uint32_t x[CPL];
            if constexpr (TEAM) {
                // The keys of phase p - 1 come from this strip and its two neighbours, which publish
                // them with the phase's tag in the low 9 bits (the offset and direction bits that
                // the DP resets here anyway); wait until every valid column shows that tag.
                const uint64_t* xr = reinterpret_cast<const uint64_t*>(d.xq + (size_t)((p - 1) & 1) * d.xw + cx);
                const uint32_t want = phase_tag(gk + p - 1);
                unsigned long long t0 = 0;
                for (int it = 0;; ++it) {
#pragma unroll
                    for (int i = 0; i < CPL / 2; ++i) {
                        const uint64_t v = ld<true>(xr + i);
                        x[2 * i] = (uint32_t)v;
                        x[2 * i + 1] = (uint32_t)(v >> 32);
                    }
                    bool ok = true;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) ok = ok && (!valid[k] || (x[k] & 0x1FFu) == want);
                    if (__all(ok)) break;
                    __builtin_amdgcn_s_sleep(1);
                    if ((it & 63) == 63) {  // bounded wait: 10 s at the 100 MHz constant clock
                        const unsigned long long now = wall_clock64();
                        if (t0 == 0) t0 = now;
                        if (now - t0 > 1000000000ull ||
                            (__hip_atomic_load(gp(d.status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                             (kStatusTimeout | kStatusPlacement))) {
                            if (lane == 0)
                                __hip_atomic_fetch_or(gp(d.status), kStatusTimeout, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                            return false;
                        }
                    }
                }
            } else {
                const uint32_t* xr = &sm.xs[(p - 1) & 1][cx];
#pragma unroll
                for (int k = 0; k < CPL; ++k) x[k] = xr[k];
            }
#pragma unroll
            for (int k = 0; k < CPL; ++k) Q[k] = valid[k] ? (x[k] & ~0x1FFu) : QINF;  // offset and tag reset
        }
        const bool cross = nx.valid && ((r1 - r0) % PF == 0);
        // The direction map groups rows by four: the dword at ((r >> 2) * db + b) * 4 holds the
        // direction byte b (4 columns, 2 bits each) of rows r & ~3 .. (r & ~3) + 3, lowest row in
        // the lowest byte.  A lane gathers its bytes of a group in registers and stores them once;
        // lanes that do not own their columns store to a dropped offset instead of branching.
        const uint32_t doff = owned && (CPL != 2 || (lane & 1) == 0) ? (uint32_t)(col0 >> 2) * 4u : kBufDrop;
        const uint32_t gbytes = (uint32_t)d.db * 4u;  // bytes per 4-row group
        uint32_t pk0 = 0, pk1 = 0;                    // CPL 8: pk1 holds the lane's second byte
        // CPL 2: a lane's two columns sit in the high half of each row byte; an even lane's byte
        // takes them to the low half and its odd neighbour's (the next two columns) on top
        auto pair_bytes = [](uint32_t pk) {
            return (pk >> 4) | (uint32_t)__builtin_amdgcn_mov_dpp((int)pk, 0xF5, 0xf, 0xf, false);  // quad_perm 1,1,3,3
        };

        auto flush = [&](int r) {  // r: the last row gathered; stores the group of row r
            const int sh = 8 * (3 - (r & 3));          // a partial group sits in the top bytes
            if constexpr (CPL == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(pair_bytes(pk0 >> sh), rdir, (int)doff,
                                                      (int)((uint32_t)(r >> 2) * gbytes), 0);
            } else if constexpr (CPL == 4) {
                __builtin_amdgcn_raw_buffer_store_b32(pk0 >> sh, rdir, (int)doff, (int)((uint32_t)(r >> 2) * gbytes), 0);
            } else {
                const v2u v = {pk0 >> sh, pk1 >> sh};
                __builtin_amdgcn_raw_buffer_store_b64(v, rdir, (int)doff, (int)((uint32_t)(r >> 2) * gbytes), 0);
            }
        };
        // EDGE: the right candidate of a column next to the image's right end, and the left one
        // of the image's column 0, saturate to all ones (the columns outside are never parents)
        uint32_t radd[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) radd[k] = valid[k] ? 10u : 0xFFFFFFFFu;
        const uint32_t ladd = valid[CPL - 1] ? 0u : 0xFFFFFFFFu;
        auto step = [&](int r, const EV& ev) {
            const uint32_t acc = row_step<EDGE>(Q, ev, radd, ladd);
            // shift the group's bytes down one and put this row's byte on top: one v_perm_b32
            // (selector bytes 0-3 pick from pk, 4-7 from acc)
            if constexpr (CPL <= 4) {
                pk0 = __builtin_amdgcn_perm(acc, pk0, 0x07030201u);
            } else {
                pk0 = __builtin_amdgcn_perm(acc, pk0, 0x06030201u);
                pk1 = __builtin_amdgcn_perm(acc, pk1, 0x07030201u);
            }
        };

        // A full block of PF rows stores its two 4-row groups together at its end: a store between
        // the prefetches would make the wait for the next block's first row cover the loads
        // issued after it (one vector memory counter for loads and stores, drained in order).
        uint32_t gk0 = 0, gk1 = 0;  // the block's first group
        auto flush_block = [&](int rb) {
            const uint32_t g0 = (uint32_t)(rb >> 2) * gbytes;
            if constexpr (CPL == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(pair_bytes(gk0), rdir, (int)doff, (int)g0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(pair_bytes(pk0), rdir, (int)doff, (int)(g0 + gbytes), 0);
            } else if constexpr (CPL == 4) {
                __builtin_amdgcn_raw_buffer_store_b32(gk0, rdir, (int)doff, (int)g0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(pk0, rdir, (int)doff, (int)(g0 + gbytes), 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b64((v2u){gk0, gk1}, rdir, (int)doff, (int)g0, 0);
                __builtin_amdgcn_raw_buffer_store_b64((v2u){pk0, pk1}, rdir, (int)doff, (int)(g0 + gbytes), 0);
            }
        };
        static_assert(PF == 8, "a block is two direction groups");

        int rb = r0;  // r0 and every block start are multiples of 4, so groups never straddle blocks
        // blocks whose prefetch targets stay inside this item
        for (; rb + 2 * PF <= r1; rb += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i) {  // the slot is refilled after its row (no register copy)
                step(rb + i, ring[i]);
                ring[i] = load_ev<TEAM>(re, soff(rb - r0 + i + PF), eoff);
                __builtin_amdgcn_sched_barrier(0);  // keep the prefetch PF rows ahead of its use
                if (i == 3) gk0 = pk0, gk1 = pk1;
            }
            flush_block(rb);
        }
        // the last full block prefetches the next item's first rows, or else this item's partial
        // tail (rows past the item's end are clamped to its last row and never stepped)
        if (rb + PF <= r1) {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                step(rb + i, ring[i]);
                ring[i] = load_ev<TEAM>(re, cross ? soffn(i) : soff(min(rb - r0 + PF + i, r1 - 1 - r0)),
                                        cross ? nx.off : eoff);
                __builtin_amdgcn_sched_barrier(0);
                if (i == 3) gk0 = pk0, gk1 = pk1;
            }
            flush_block(rb);
            rb += PF;
        }
        // the rows of a partial last phase (the next item then loads its own first rows)
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            if (rb + i < r1) {
                step(rb + i, ring[i]);
                if ((i & 3) == 3 || rb + i == r1 - 1) flush(rb + i);
            }
        }

        // phase end: publish the last row of the owned columns and their ancestor offsets
        if (owned) {
            if constexpr (TEAM) {
                uint32_t* xw = d.xq + (size_t)(p & 1) * d.xw + col0;
                const uint32_t tag = phase_tag(gk + p);
#pragma unroll
                for (int k = 0; k < CPL; ++k) *gp(xw + k) = (Q[k] & ~0x1FFu) | tag;
            } else {
                uint32_t* xw = &sm.xs[p & 1][col0];
#pragma unroll
                for (int k = 0; k < CPL; ++k) xw[k] = Q[k];
            }
            if (p > 0) {
                const int n = r1 - r0;
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if (valid[k]) *gp(d.anc + (size_t)p * d.W + col0 + k) = (int8_t)((int)((Q[k] >> 2) & 127u) - n);
            }
        }
        if (r1 == d.H) {  // last row: leftmost argmin of M over the owned columns
            unsigned long long key = ~0ull;
            if (owned) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const unsigned long long kk = ((unsigned long long)(Q[k] >> 9) << 32) | (unsigned)(col0 + k);
                    if (valid[k] && kk < key) key = kk;
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long o = __shfl_xor(key, off, 64);
                key = o < key ? o : key;
            }
            if (lane == 0 && key != ~0ull) __hip_atomic_fetch_min(gp(d.amin), key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return true;
    }

    // Seams k_begin .. k_end-1 of one image (the image has W - k_begin columns on entry).  With a
    // deadline (device wall clock; one workgroup only) it stops after the first seam that ends
    // past it.  Returns the number of seams removed in total (k_begin + the seams of this call).
    template <bool TEAM>
    static __device__ __forceinline__ int carve_seams(const Img& d, int rank, int G, Smem& sm, int k_begin, int k_end,
                                                      unsigned& epoch, unsigned long long deadline) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        // waves are numbered across the team first, so a phase's strips land on different compute
        // units (one DP wave per SIMD) before any workgroup takes a second one
        const int TW = G * NW, tw = wv * G + rank;
        const int rpw = (d.H + TW - 1) / TW;
        const int ra = min(d.H, tw * rpw), rb = min(d.H, ra + rpw);  // rows this wave owns
        const int H = d.H, P = d.P;
        GAS Ctl* ctl = gp(reinterpret_cast<Ctl*>(d.amin));
        const bool timer = rank == 0 && threadIdx.x == 0;  // one clock reader per image
        unsigned long long tm0 = 0, tm1 = 0, tm2 = 0;
        for (int k = k_begin; k < k_end; ++k) {
            const int w = d.W - k;
            if (timer) tm0 = wall_clock64();
            // ---- DP sweep, phase by phase (a3), and the bottom-row argmin (a4)
            const int nstr = (w + S - 1) / S;
            const int nsw = tw < nstr ? (nstr - tw + TW - 1) / TW : 0;  // strips of this wave per phase
            EV ring[PF];
            bool preloaded = false;
            int rovc = 0;
            // no phase end of this seam is known yet; the DP's barriers order this reset before
            // any walker of this seam reads it, and after every walker of the previous seam
            if (threadIdx.x == 0) sm.chain = 0x7fffffff;
            for (int p = 0; p < P; ++p) {
                for (int j = 0; j < nsw; ++j) {
                    const int t = tw + j * TW;
                    const bool last = (p == P - 1) && (j == nsw - 1);
                    const int pn = j + 1 < nsw ? p : p + 1;
                    const int tn = j + 1 < nsw ? t + TW : tw;
                    const Next nx = make_next(d, w, pn, tn, lane, !last);
                    const int base = t * S - KR;
                    const bool ok = (base < 0 || base + WIN > w)
                                        ? dp_item<true, TEAM>(d, sm, w, p, t, lane, ring, preloaded, nx, k * P, rovc)
                                        : dp_item<false, TEAM>(d, sm, w, p, t, lane, ring, preloaded, nx, k * P, rovc);
                    if (!ok) return k;
                    preloaded = nx.valid && ((min(H, p * KR + KR) - p * KR) % PF == 0);
                }
                // one workgroup exchanges phase ends through LDS behind a barrier; a team's waves
                // wait only for the tagged keys of their neighbours (in dp_item)
                if constexpr (!TEAM) __syncthreads();
            }
            // the directions, ancestor offsets and argmin of every phase are complete past here
            if constexpr (TEAM) {
                if (!team_sync<TEAM>(d, epoch, G, &sm.flag)) return k;
            }
            if (timer) tm1 = wall_clock64();
            const unsigned long long key = __hip_atomic_load(gp(d.amin), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int jstar = min(max((int)(key & 0xffffffffu), 0), w - 1);
            if (rank == 0 && threadIdx.x == 0 && d.costs_out) *gp(d.costs_out + k) = (long long)(key >> 32);
            // ---- backtrack (a5): wave 0 hops from phase end to phase end and publishes the seam
            // column at every phase end in LDS as soon as it is known; the waves walk their phases'
            // rows from LDS windows of the direction map as their phase ends become known.  A phase
            // end lies within KR columns of the one below it, so a round loads the ancestor offsets
            // of CH phases at once (the 512 bytes of each row around the current column, two dwords
            // per lane, into LDS that the DP no longer uses) and lane 0 takes CH hops from there:
            // one memory round trip per CH hops instead of one per hop.
            if (wv == 0) {
                constexpr int CH = 252 / KR + 1;  // h * KR + 3 < 256 for every hop h of a round
                static_assert(CH * 128 <= 2 * kLdsExchangeMaxW, "hop windows fit the exchange rows");
                uint32_t* cw = &sm.xs[0][0];
                const __amdgpu_buffer_rsrc_t ranc = make_rsrc(d.anc, ((uint32_t)P * (uint32_t)d.W + 3u) & ~3u);
                int j = jstar;
                if (lane == 0) {
                    sm.jend[P - 1] = j;
                    __hip_atomic_store(&sm.chain, P - 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                for (int p = P - 1; p >= 1; p -= CH) {
                    const int m = min(CH, p);
                    uint32_t v[CH][2];
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        // byte window [o, o + 512) of phase p - h's row, o = row + j - 256 rounded
                        // down to a dword; dwords before the array are dropped
                        const int o = (p - h) * d.W + j - 256;
                        const int oa = o >= 0 ? o & ~3 : -((-o + 3) & ~3);
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int bo = oa + 4 * (lane + 64 * q);
                            v[h][q] = buf_ld32<TEAM>(ranc, h < m && bo >= 0 ? (uint32_t)bo : kBufDrop);
                        }
                    }
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        cw[h * 128 + lane] = v[h][0];
                        cw[h * 128 + 64 + lane] = v[h][1];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (lane == 0) {
                        const uint8_t* cb = reinterpret_cast<const uint8_t*>(cw);
                        const int j0 = j;
                        for (int h = 0; h < m; ++h) {
                            const int o = (p - h) * d.W + j0 - 256;
                            const int oa = o >= 0 ? o & ~3 : -((-o + 3) & ~3);
                            j = min(max(j + (int)(int8_t)cb[h * 512 + (p - h) * d.W + j - oa], 0), w - 1);
                            sm.jend[p - 1 - h] = j;
                            __hip_atomic_store(&sm.chain, p - 1 - h, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                    j = __builtin_amdgcn_readfirstlane(j);  // lane 0's column, after its LDS reads
                    __builtin_amdgcn_wave_barrier();
                }
            }
            // Each wave owns an equal range of rows [ra, rb) for the walk's output, the removal and
            // the band update.  It walks every phase its range touches (bottom phase first: phase
            // ends become known from the bottom up) and keeps the rows of its range.
            const __amdgpu_buffer_rsrc_t rdw = make_rsrc(d.dirs, (uint32_t)((H + 3) >> 2) * (uint32_t)d.db * 4u);
            for (int p = (rb - 1) / KR; ra < rb && p >= ra / KR; --p) {
                const int r0 = p * KR, r1 = min(H, r0 + KR), n = r1 - r0;
                const int ia = max(ra, r0) - r0, ib = min(rb, r1) - r0;  // this wave's rows of the phase
                while (__hip_atomic_load(&sm.chain, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) > p)
                    __builtin_amdgcn_s_sleep(1);
                const int je = sm.jend[p];
                // the walk stays within KR columns of je: direction bytes cb0 .. cb0 + GW - 1 of
                // every 4-row group of the phase, kept in LDS as [group][byte]
                constexpr int GW = 4 * WD;
                const int cb0 = max(0, je - KR) >> 2;
                uint32_t* win = sm.win[wv];
                {
                    // lane q < GW loads byte-dword cb0 + q of every 4-row group the walk reads
                    // (groups ia/4 .. of the phase): one buffer load per group at the same per-lane
                    // offset and a scalar group offset, all issued before the LDS writes (one
                    // memory round trip); lanes past the window or the map load nothing
                    constexpr int GK = KR / 4;
                    const int g0 = ia >> 2, ng = (n + 3) >> 2;  // groups holding rows ia .. n-1
                    const uint32_t lo = lane < GW && cb0 + lane < d.db ? (uint32_t)(cb0 + lane) * 4u : kBufDrop;
                    const uint32_t gb = (uint32_t)d.db * 4u;
                    uint32_t v[GK];
#pragma unroll
                    for (int j = 0; j < GK; ++j)
                        v[j] = j >= g0 && j < ng ? __builtin_amdgcn_raw_buffer_load_b32(
                                                       rdw, (int)lo, (int)((uint32_t)((r0 >> 2) + j) * gb), TEAM ? 16 : 0)
                                                 : 0u;
                    if (lane < GW) {
#pragma unroll
                        for (int j = 0; j < GK; ++j)
                            if (j >= g0 && j < ng) win[j * GW + lane] = v[j];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int s = je, mys = 0;
                for (int i = n - 1; i >= ia; --i) {
                    if (lane == i) mys = s;
                    if (i > 0) {
                        const int q = min(max((s >> 2) - cb0, 0), GW - 1);
                        const uint32_t wd = win[(i >> 2) * GW + q];
                        s += (int)((wd >> ((i & 3) * 8 + (s & 3) * 2)) & 3u) - 1;
                        s = min(max(s, 0), w - 1);
                    }
                }
                if (lane >= ia && lane < ib) {
                    *gp(d.seam + r0 + lane) = mys;
                    if (d.seams_out) *gp(d.seams_out + (size_t)k * H + r0 + lane) = mys;
                }
                __builtin_amdgcn_wave_barrier();
                if (!d.mode) {
                    // ---- removal (a6) of this wave's rows: image bytes and energy plane.  A row is
                    // only ever written by the wave owning it (this shift, the band update below and
                    // the final compaction) or by the earlier energy pass, so plain loads see its
                    // current bytes even in a team.  With min-side removal the shorter side of the
                    // row moves: pixels right of the seam one column left, or pixels left of it one
                    // column right with the row's start offset advanced by one.
                    const int rof = lane >= ia && lane < ib ? *gp(d.ro + r0 + lane) : 0;
                    // row i's shift: the shorter side with min-side removal, else the right part
                    auto right_side = [&](int i) {
                        const int si = __builtin_amdgcn_readlane(mys, i);
                        return d.minside && si < w - 1 - si;
                    };
                    auto segs = [&](int i, bool R, SSeg& gi, SSeg& ge) {
                        const int si = __builtin_amdgcn_readlane(mys, i);
                        const int o = __builtin_amdgcn_readlane(rof, i);
                        // rows of wk and of the energy plane start on 64-byte boundaries
                        uint8_t* row = d.wk + (long long)(r0 + i) * d.wp + (long long)o * d.C;
                        uint8_t* er = reinterpret_cast<uint8_t*>(d.e + (size_t)(r0 + i) * d.ep + o);
                        if (R) {
                            gi = sseg<true>(row, row + (long long)si * d.C, d.C);
                            ge = sseg<true>(er, er + 2 * si, 2);
                            if (lane == 0) *gp(d.ro + r0 + i) = o + 1;
                        } else {
                            gi = sseg<false>(row + (long long)si * d.C, row + (long long)(w - 1) * d.C, d.C);
                            ge = sseg<false>(er + 2 * si, er + 2 * (w - 1), 2);
                        }
                    };
#pragma unroll 1
                    for (int i = ia; i < ib; i += 2) {  // two rows per memory round trip
                        const bool two = i + 1 < ib;
                        const bool ra = right_side(i), rb = two && right_side(i + 1);
                        SSeg a0, a1, b0, b1;
                        segs(i, ra, a0, a1);
                        if (two) {
                            segs(i + 1, rb, b0, b1);
                        } else {
                            b0 = a0; b0.n = 0;
                            b1 = a1; b1.n = 0;
                        }
                        if (ra) {
                            if (rb) shift_rows2_wave<1, true, true>(a0, a1, b0, b1, lane);
                            else shift_rows2_wave<1, true, false>(a0, a1, b0, b1, lane);
                        } else {
                            if (rb) shift_rows2_wave<1, false, true>(a0, a1, b0, b1, lane);
                            else shift_rows2_wave<1, false, false>(a0, a1, b0, b1, lane);
                        }
                    }
                }
            }
            if (!team_sync<TEAM>(d, epoch, G, &sm.flag)) return k;
            if (timer) tm2 = wall_clock64();
            if (d.mode) break;
            if (rank == 0 && threadIdx.x == 0)
                __hip_atomic_store(gp(d.amin), ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // ---- band energy (a2): only the new columns s-1 and s of each row changed.  Buffer
            // loads (sc1 in a team: the rows above and below were shifted by other workgroups) at
            // 32-bit offsets; a lane past the wave's rows reads row ra and stores nothing.
            const int w2 = w - 1;
            const __amdgpu_buffer_rsrc_t rwk = make_rsrc(d.wk, (uint32_t)H * (uint32_t)d.wp);
            const __amdgpu_buffer_rsrc_t rsm = make_rsrc(d.seam, (uint32_t)H * 4u);
            const __amdgpu_buffer_rsrc_t rof = make_rsrc(d.ro, (uint32_t)H * 4u);
            for (int rc = ra; rc < rb; rc += 64) {
                const int r = rc + lane < rb ? rc + lane : ra;
                const int ru = r > 0 ? r - 1 : 0, rd = r + 1 < H ? r + 1 : H - 1;
                const int s = min(max((int)buf_ld32<TEAM>(rsm, (uint32_t)r * 4u), 0), w - 1);
                const int o = (int)buf_ld32<TEAM>(rof, (uint32_t)r * 4u);
                const uint32_t br = (uint32_t)r * (uint32_t)d.wp + (uint32_t)(o * d.C);
                const uint32_t bu = (uint32_t)ru * (uint32_t)d.wp + buf_ld32<TEAM>(rof, (uint32_t)ru * 4u) * (uint32_t)d.C;
                const uint32_t bd = (uint32_t)rd * (uint32_t)d.wp + buf_ld32<TEAM>(rof, (uint32_t)rd * 4u) * (uint32_t)d.C;
                const uint32_t e0 = energy_buf<TEAM>(rwk, br, bu, bd, w2, d.C, s - 1);
                const uint32_t e1 = energy_buf<TEAM>(rwk, br, bu, bd, w2, d.C, s);
                if (rc + lane < rb) {
                    uint16_t* er = d.e + (size_t)r * d.ep + o;
                    if (s - 1 >= 0 && s - 1 < w2) *gp(er + s - 1) = (uint16_t)e0;
                    if (s < w2) *gp(er + s) = (uint16_t)e1;
                }
            }
            // a team's time budget: its first member decides before the seam's last barrier, every
            // member reads the decision after it
            if (deadline && G > 1 && k + 1 < k_end && rank == 0 && threadIdx.x == 0)
                __hip_atomic_store(&ctl->stop, wall_clock64() >= deadline ? 1u : 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            if (!team_sync<TEAM>(d, epoch, G, &sm.flag)) return k;
            if (deadline && G > 1 && k + 1 < k_end && __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) k_end = k + 1;
            if (timer) {
                const unsigned long long tm3 = wall_clock64();
                ctl->t_stage[0] += tm1 - tm0;
                ctl->t_stage[1] += tm2 - tm1;
                ctl->t_stage[2] += tm3 - tm2;
            }
            if (deadline && G == 1 && k + 1 < k_end) {  // one decision for the whole workgroup
                if (threadIdx.x == 0) sm.stop = wall_clock64() >= deadline;
                __syncthreads();
                const int stop = sm.stop;
                __syncthreads();
                if (stop) k_end = k + 1;
            }
        }
        // ---- after the last seam, the carved rows go from wk (each from its start offset) to img
        if (!d.mode && k_end == d.W - d.target_w && k_end > k_begin) {
            const int nb = d.target_w * d.C;
            for (int rc = ra; rc < rb; rc += 64) {
                const int n = min(64, rb - rc);
                const int rof = lane < n ? *gp(d.ro + rc + lane) : 0;
#pragma unroll 1
                for (int i = 0; i < n; ++i) {
                    const int o = __builtin_amdgcn_readlane(rof, i);
                    copy_bytes_wave(d.img + (long long)(rc + i) * d.pitch, d.wk + (long long)(rc + i) * d.wp + (long long)o * d.C,
                                    nb, lane);
                }
            }
            team_sync<TEAM>(d, epoch, G, &sm.flag);
        }
        return k_end;
    }

    // Carve one image, or (max_seams > 0) continue it by at most max_seams seams.
    static __device__ __forceinline__ void carve_image(const Img& d, int rank, int G, Smem& sm, int max_seams,
                                                       unsigned long long deadline = 0) {
        GAS Ctl* ctl = gp(reinterpret_cast<Ctl*>(d.amin));
        const int nseams = d.mode ? 1 : d.W - d.target_w;
        const int k0 = max_seams > 0 ? (int)ctl->done : 0;
        const int k1 = max_seams > 0 ? min(nseams, k0 + max_seams) : nseams;
        if (k0 >= k1) return;
        if (rank == 0 && threadIdx.x == 0 && k0 == 0) ctl->t_begin = wall_clock64();
        // a call that continues a carve (step mode) starts from the barrier count the previous
        // calls left behind, so a team's barrier counter never has to be reset between launches
        unsigned epoch = max_seams > 0 ? __hip_atomic_load(&ctl->ebase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        int kd = k0;  // seams removed in total when this call ends
        const bool team = G > 1 || d.W > kLdsExchangeMaxW;
        if (team) {
            if (max_seams > 0) {
                // keys published in an earlier step may carry any tag; the members clear the
                // exchange rows (ordered before every DP by the barrier below)
                for (int x = rank * NT + (int)threadIdx.x; x < 2 * d.xw; x += G * NT) *gp(d.xq + x) = 0u;
            }
            // every member records its XCD; a team spread over several XCDs would not see each
            // other's stores through sc1 loads, so such an image is flagged instead of carved
            if (threadIdx.x == 0) __hip_atomic_fetch_or(&ctl->xmask, 1u << (xcc_id() & 31), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (!team_sync<true>(d, epoch, G, &sm.flag)) return;
            const unsigned m = __hip_atomic_load(&ctl->xmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__popc(m) != 1) {
                if (threadIdx.x == 0)
                    __hip_atomic_fetch_or(gp(d.status), kStatusPlacement, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            kd = carve_seams<true>(d, rank, G, sm, k0, k1, epoch, deadline);
        } else {
            kd = carve_seams<false>(d, rank, G, sm, k0, k1, epoch, deadline);
        }
        __syncthreads();
        if (rank == 0 && threadIdx.x == 0) {
            ctl->done = (unsigned)kd;
            if (kd == nseams) ctl->t_end = wall_clock64();
            if (max_seams > 0) {  // every member ended this call at the same barrier count
                ctl->ebase = epoch;
                ctl->xmask = 0;
                ctl->stop = 0;
            }
        }
    }
};

template <int CPL, int KR, int NT>
__global__ __launch_bounds__(NT, 4) void carve_single_kernel(Img d, int xcd) {
    using CV = Carver<CPL, KR, NT>;
    __shared__ typename CV::Smem sm;
    // Team members are blocks xcd, xcd + 8, xcd + 16, ...: workgroups are dispatched to the 8 XCDs
    // round-robin by block index, so they share XCD `xcd`'s L2; the other blocks exit at once.
    if ((int)(blockIdx.x & 7) != xcd) return;
    CV::carve_image(d, blockIdx.x >> 3, d.G, sm, 0);
}

// Batched carve: block b is member blk[b].y of team blk[b].x; team t carves the images
// team_imgs[teams[t].x .. teams[t].x + teams[t].y) one after another.
template <int CPL, int KR, int NT>
__global__ __launch_bounds__(NT, 4) void carve_batch_kernel(const Img* __restrict__ imgs, const int2* __restrict__ blk,
                                                         const int2* __restrict__ teams,
                                                         const int* __restrict__ team_imgs) {
    using CV = Carver<CPL, KR, NT>;
    __shared__ typename CV::Smem sm;
    const int2 me = blk[blockIdx.x];
    if (me.x < 0) return;
    const int2 tr = teams[me.x];
    for (int i = 0; i < tr.y; ++i) {
        const Img d = imgs[team_imgs[tr.x + i]];
        CV::carve_image(d, me.y, d.G, sm, 0);
        __syncthreads();
    }
}

// Step-wise carve (serving): each image of the slot table advances by at most max_seams seams and
// reports how many seams it has removed in total (-1 on a device error, -2 for an empty slot).
// Without a plan block b carves slot b alone; with one, block b is member plan[b].y of the team of
// plan[b].z workgroups that carves slot plan[b].x (-1: no work), the members of a team on one XCD.
// The table is a device array of descriptors written by slot_write_kernel.
template <int CPL, int KR, int NT>
__global__ __launch_bounds__(NT, 4) void carve_steps_kernel(const Img* __restrict__ table, int n, int max_seams,
                                                            unsigned long long budget_ticks,
                                                            int* __restrict__ progress, const int4* __restrict__ plan) {
    using CV = Carver<CPL, KR, NT>;
    __shared__ typename CV::Smem sm;
    int slot = (int)blockIdx.x, rank = 0, G = 1;
    if (plan) {
        const int4 p = plan[blockIdx.x];
        slot = p.x;
        rank = p.y;
        G = p.z;
    }
    if (slot < 0 || slot >= n) return;
    const Img d = table[slot];
    if (d.H == 0) {
        if (rank == 0 && threadIdx.x == 0 && progress) progress[slot] = -2;
        return;
    }
    // a time budget (device wall clock ticks) ends the image's share after the seam that crosses
    // it, so a step's workgroups stay busy for about the same time
    CV::carve_image(d, rank, G, sm, max_seams, budget_ticks ? wall_clock64() + budget_ticks : 0ull);
    __syncthreads();
    if (rank == 0 && threadIdx.x == 0 && progress) {
        const GAS Ctl* ctl = gp(reinterpret_cast<const Ctl*>(d.amin));
        progress[slot] = (ctl->status & (kStatusTimeout | kStatusPlacement)) ? -1 : (int)ctl->done;
    }
}

// Slot management: write (or clear) one descriptor of the slot table.
__global__ void slot_write_kernel(Img* table, int slot, Img d) { table[slot] = d; }

// Unpack the 2-bit direction map into bytes (row 0 has no parent: 1).
__global__ void unpack_dirs_kernel(Img d, uint8_t* __restrict__ out) {
    const int y = blockIdx.y;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < d.W; x += gridDim.x * blockDim.x) {
        uint8_t v = 1;
        if (y > 0) v = (*gp(d.dirs + ((size_t)(y >> 2) * d.db + (x >> 2)) * 4 + (y & 3)) >> ((x & 3) * 2)) & 3u;
        *gp(out + (size_t)y * d.W + x) = v;
    }
}

// ----------------------------------------------------------------------------------------------
// Seam insertion (image enlargement).
//
// Original columns of seams recorded during removal: one thread per row keeps a Fenwick tree over
// the row's columns still present (1 each) and finds seam j's column as the (s+1)-th present one,
// then takes it out.  tree: (W + 1) * H int32, entry i of row r at tree[i * H + r] (neighbouring
// threads touch neighbouring words).
__global__ void seam_origins_kernel(const int32_t* __restrict__ seams, int k, int H, int W, int32_t* __restrict__ tree,
                                    int32_t* __restrict__ orig) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= H) return;
    int32_t* T = tree + r;
    const size_t st = (size_t)H;
    for (int i = 1; i <= W; ++i) *gp(T + i * st) = i & -i;
    int top = 1;
    while ((top << 1) <= W) top <<= 1;
    for (int j = 0; j < k; ++j) {
        int rem = min(max(*gp(seams + (size_t)j * H + r), 0), W - 1 - j) + 1;
        int pos = 0;  // the largest index whose prefix count is below rem
        for (int step = top; step > 0; step >>= 1) {
            const int nx = pos + step;
            if (nx <= W) {
                const int v = *gp(T + nx * st);
                if (v < rem) {
                    pos = nx;
                    rem -= v;
                }
            }
        }
        *gp(orig + (size_t)j * H + r) = pos;  // 0-based column of the (s+1)-th present one
        for (int i = pos + 1; i <= W; i += i & -i) *gp(T + i * st) -= 1;
    }
}

// Widened rows: one workgroup per row marks the seams' original columns in an LDS bitmap, counts
// the marks per thread chunk, scans the counts, and writes every pixel at its column plus the
// number of marks left of it, followed by the new pixel ((a + b + 1) >> 1 with the right
// neighbour; the pixel itself at the last column) where a column is marked.
constexpr int kInsertThreads = 256;
constexpr int kInsertMaxW = kInsertMaxWidth;  // the row bitmap lives in LDS
__global__ __launch_bounds__(kInsertThreads) void insert_seams_kernel(const uint8_t* __restrict__ img, int W, int C,
                                                                    long long pitch, int H, int k,
                                                                    const int32_t* __restrict__ orig,
                                                                    uint8_t* __restrict__ out, long long out_pitch) {
    __shared__ uint32_t bm[kInsertMaxW / 32];
    __shared__ int part[kInsertThreads];
    const int r = blockIdx.x, t = threadIdx.x;
    const int nwords = (W + 31) >> 5;
    for (int i = t; i < nwords; i += kInsertThreads) bm[i] = 0u;
    __syncthreads();
    for (int j = t; j < k; j += kInsertThreads) {
        const int c = min(max(*gp(orig + (size_t)j * H + r), 0), W - 1);
        atomicOr(&bm[c >> 5], 1u << (c & 31));
    }
    __syncthreads();
    const int wpt = (nwords + kInsertThreads - 1) / kInsertThreads;  // bitmap words per thread
    const int w0 = min(t * wpt, nwords), w1 = min(w0 + wpt, nwords);
    int cnt = 0;
    for (int i = w0; i < w1; ++i) cnt += __popc(bm[i]);
    part[t] = cnt;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int i = 0; i < kInsertThreads; ++i) {
            const int v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int before = part[t];  // marks left of this thread's first column
    const uint8_t* row = img + (long long)r * pitch;
    uint8_t* o = out + (long long)r * out_pitch;
    for (int c = w0 * 32; c < min(w1 * 32, W); ++c) {
        const int pos = c + before;
        for (int ch = 0; ch < C; ++ch) *gp(o + (long long)pos * C + ch) = *gp(row + (long long)c * C + ch);
        if ((bm[c >> 5] >> (c & 31)) & 1u) {
            const int cr = c + 1 < W ? c + 1 : c;
            for (int ch = 0; ch < C; ++ch) {
                const int a = *gp(row + (long long)c * C + ch), b = *gp(row + (long long)cr * C + ch);
                *gp(o + (long long)(pos + 1) * C + ch) = (uint8_t)((a + b + 1) >> 1);
            }
            ++before;
        }
    }
}

// Launchers of the carve kernel variants (the table of shapes: SC_VARIANTS in sc_internal.h).
hipError_t launch_carve_single(const Img& d, int v, int G, int xcd, hipStream_t st) {
    switch (v) {
#define X(id, c, k, t) \
    case id: hipLaunchKernelGGL((carve_single_kernel<c, k, t>), dim3(8 * G), dim3(t), 0, st, d, xcd & 7); break;
        SC_VARIANTS(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_carve_batch(const Img* imgs, const int2* blk, const int2* teams, const int* ti, int nb, int v,
                              hipStream_t st) {
    switch (v) {
#define X(id, c, k, t) \
    case id: hipLaunchKernelGGL((carve_batch_kernel<c, k, t>), dim3(nb), dim3(t), 0, st, imgs, blk, teams, ti); break;
        SC_VARIANTS(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_carve_steps(const Img* table, int n, int v, int max_seams, unsigned long long budget_ticks,
                              int* progress, const int4* plan, int nblocks, hipStream_t st) {
    const int nb = plan ? nblocks : n;
    switch (v) {
#define X(id, c, k, t)                                                                                        \
    case id:                                                                                                  \
        hipLaunchKernelGGL((carve_steps_kernel<c, k, t>), dim3(nb), dim3(t), 0, st, table, n, max_seams, budget_ticks, \
                           progress, plan);                                                                        \
        break;
        SC_VARIANTS(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


hipError_t launch_slot_write(Img* table, int slot, const Img& d, hipStream_t st) {
    hipLaunchKernelGGL(slot_write_kernel, dim3(1), dim3(1), 0, st, table, slot, d);
    return hipGetLastError();
}

hipError_t launch_seam_origins(const int32_t* seams, int k, int H, int W, int32_t* tree, int32_t* orig,
                               hipStream_t st) {
    hipLaunchKernelGGL(seam_origins_kernel, dim3((H + 63) / 64), dim3(64), 0, st, seams, k, H, W, tree, orig);
    return hipGetLastError();
}

hipError_t launch_insert_seams(const uint8_t* img, int H, int W, int C, long long pitch, int k, const int32_t* orig,
                               uint8_t* out, long long out_pitch, hipStream_t st) {
    if (W > kInsertMaxW) return hipErrorInvalidValue;
    hipLaunchKernelGGL(insert_seams_kernel, dim3(H), dim3(kInsertThreads), 0, st, img, W, C, pitch, H, k, orig, out,
                       out_pitch);
    return hipGetLastError();
}

int carve_blocks_per_cu(int v) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (v) {
#define X(id, c, k, t) \
    case id: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, carve_batch_kernel<c, k, t>, t, 0); break;
        SC_VARIANTS(X)
#undef X
        default: break;
    }
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_energy_i32(const uint8_t* img, int H, int W, int C, long long pitch, int32_t* out, hipStream_t st) {
    dim3 grid((W + 255) / 256, H);
    hipLaunchKernelGGL(energy_i32_kernel, grid, dim3(256), 0, st, img, H, W, C, pitch, out);
    return hipGetLastError();
}

hipError_t launch_prepare_single(const Img& d, hipStream_t st) {
    const int tiles = ((d.W + kTileCols - 1) / kTileCols) * ((d.H + kTileRows - 1) / kTileRows);
    const int blocks = tiles < 4096 ? tiles : 4096;
    hipLaunchKernelGGL(prepare_single_kernel, dim3(blocks), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_prepare_from_i32(const Img& d, const int32_t* e, hipStream_t st) {
    dim3 grid((d.W + 255) / 256, d.H);
    hipLaunchKernelGGL(prepare_from_i32_kernel, grid, dim3(256), 0, st, d, e);
    return hipGetLastError();
}

hipError_t launch_prepare_batch(const Img* imgs, int n, int max_rows, hipStream_t st) {
    // workgroups per image: enough for the tiles of a tall image (each takes every per-th tile)
    const int chunks = (max_rows + kTileRows - 1) / kTileRows;
    const int per = chunks < 64 ? chunks : 64;
    hipLaunchKernelGGL(prepare_batch_kernel, dim3(per, n), dim3(256), 0, st, imgs, n);
    return hipGetLastError();
}

hipError_t launch_unpack_dirs(const Img& d, uint8_t* out, hipStream_t st) {
    dim3 grid((d.W + 255) / 256, d.H);
    hipLaunchKernelGGL(unpack_dirs_kernel, grid, dim3(256), 0, st, d, out);
    return hipGetLastError();
}

hipError_t launch_remove_seam(uint8_t* img, int H, int W, int C, long long pitch, const int32_t* seam,
                              hipStream_t st) {
    const int waves = H < 4096 ? H : 4096;
    hipLaunchKernelGGL(remove_seam_kernel, dim3((waves + 3) / 4), dim3(256), 0, st, img, H, W, C, pitch, seam);
    return hipGetLastError();
}

hipError_t launch_transpose(const uint8_t* src, int H, int W, int C, long long sp, uint8_t* dst, long long dp,
                            hipStream_t st) {
    dim3 grid((W + 63) / 64, (H + 63) / 64);
    switch (C) {
        case 1: hipLaunchKernelGGL(transpose_kernel<1>, grid, dim3(256), 0, st, src, H, W, sp, dst, dp); break;
        case 2: hipLaunchKernelGGL(transpose_kernel<2>, grid, dim3(256), 0, st, src, H, W, sp, dst, dp); break;
        case 3: hipLaunchKernelGGL(transpose_kernel<3>, grid, dim3(256), 0, st, src, H, W, sp, dst, dp); break;
        case 4: hipLaunchKernelGGL(transpose_kernel<4>, grid, dim3(256), 0, st, src, H, W, sp, dst, dp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Fixed scratch of the allocation-free carve (sc_carve_noalloc): a file-scope device array, one
// copy per GPU, held until the process ends.  In host code the array's name is only a host-side
// stand-in for it; the device address of each GPU's copy is looked up once per device with that
// device current and kept, and only that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
    static std::mutex mu;
    static void* addr[kNoAllocMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

__global__ void copy_status_kernel(const unsigned* __restrict__ src, uint32_t* __restrict__ dst) { *dst = *src; }

hipError_t launch_copy_status(const unsigned* src, uint32_t* dst, hipStream_t st) {
    hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(1), 0, st, src, dst);
    return hipGetLastError();
}

}  // namespace sc
