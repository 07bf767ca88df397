// Object removal with a mask (sec. "Object Removal" among the applications of the paper) on
// gfx950: the pixels of a binary mask receive a very large negative energy, so every seam runs
// through the object while any of it is left; the seams are removed from the image and from the
// mask alike until no masked pixel remains.
//
// The masked energy of a pixel is its e1 energy minus B = h*510*C + 1 under the mask (h = rows of
// the carved frame).  B exceeds the e1 energy of any whole seam, so over the paths reaching a
// cell in row i (all of i+1 pixels) the masked cost E - B*m orders exactly like the pair
// (q, E) with q = i+1-m, the number of unmasked pixels, compared first: the DP carries q and E as
// one 64-bit key (q in the high word; E << 9 | ancestor offset in the low word, with the
// direction tag in bits 7-8 while the three parents are compared) and never forms the negative
// sum.  Ties fall to the leftmost parent and the leftmost last-row column, as in the plain carve,
// so the seam is the oracle's minimum of E - B*m.
//
// One 1024-thread workgroup carves one image (thread t owns columns [CPL*t, CPL*t + CPL)), in
// the row-synchronous style of the forward-energy kernel: the e1 energy of every cell is computed
// from the current pixels while the DP sweeps the rows (three pixel rows around the cell), so
// there is no energy plane to keep up to date; neighbour keys cross threads through LDS with one
// barrier per row; the 2-bit direction map and per-phase ancestor offsets drive the backtrack;
// the removal shifts the pixel row and the mask row of every seam row in one pass.
#include "sc_device.h"

namespace sc {
namespace obj {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
constexpr int K = kFwdPhaseRows;  // rows per phase: the ancestor offset stays in [4, 124]
constexpr int GK = K / 4;         // 4-row direction groups per phase
constexpr int WD = 32;            // window dwords per group: columns je-59 .. je+59
constexpr int PMAX = (kFwdMaxH + K - 1) / K;
constexpr int ANC_LDS = 64 * 1024;  // phase ancestors kept in LDS up to this many bytes
constexpr unsigned long long INF = ~0ull;
static_assert(K % 4 == 0 && K <= 63, "phase shape");

struct Smem {
    unsigned long long xa[2][NT + 1];  // first column key of thread t at [t]
    unsigned long long xb[2][NT + 1];  // last column key of thread t at [t + 1]
    uint32_t win[NW][GK * WD];
    int jend[PMAX];  // seam column at the last row of every phase
    unsigned long long red[NW];
    int cnt[NW];
    int left;  // masked pixels still in the image
};

__device__ __forceinline__ unsigned long long min64(unsigned long long a, unsigned long long b) { return b < a ? b : a; }

// Number of nonzero bytes of v.
__device__ __forceinline__ int nonzero_bytes(uint32_t v) {
    return __popc((((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u);
}

template <int C, int CPL>
struct Carver : PixRow<C, CPL> {
    using Row = PixRow<C, CPL>;
    using Row::load_row;
    using Row::pixels;
    static constexpr int NDW = Row::NDW;
    static constexpr int PF = 4;  // rows of pixels and mask loaded ahead
    static constexpr int MD = CPL / 4;           // mask dwords per thread and row
    static_assert(PF % 4 == 0, "direction groups");

    static __device__ __forceinline__ void load_mask(uint32_t (&m)[MD], __amdgpu_buffer_rsrc_t r, uint32_t mo,
                                                     uint32_t soff) {
#pragma unroll
        for (int q = 0; q < MD; ++q) m[q] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(mo + 4u * q), (int)soff, 0);
    }

    static __device__ __forceinline__ void carve(const ObjImg& d, Smem& sm, uint8_t* anc_lds) {
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        const int H = d.H, W = d.W, j0 = t * CPL;
        GAS ObjCtl* ctl = gp(d.ctl);
        if (t == 0) ctl->t_begin = wall_clock64();
        const long long bias = (long long)H * 510 * C + 1;

        // ---- masked pixels of the frame (any nonzero byte marks a pixel)
        {
            int cnt = 0;
#pragma unroll 1
            for (int r = wv; r < H; r += NW) {
                const uint8_t* mr = d.mk + (long long)r * d.mp;
                for (int x = lane * 4; x < W; x += 256) {
                    uint32_t v = *gp(reinterpret_cast<const uint32_t*>(mr + x));
                    if (x + 4 > W) v &= (1u << (8 * (W - x))) - 1u;
                    cnt += nonzero_bytes(v);
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
            if (lane == 0) sm.cnt[wv] = cnt;
            __syncthreads();
            if (t == 0) {
                int s = 0;
                for (int x = 0; x < NW; ++x) s += sm.cnt[x];
                sm.left = s;
            }
            __syncthreads();
        }

        const __amdgpu_buffer_rsrc_t rwk = make_rsrc(d.wk, (uint32_t)H * (uint32_t)d.wp + (uint32_t)kFwdSlack);
        const __amdgpu_buffer_rsrc_t rmk = make_rsrc(d.mk, (uint32_t)H * (uint32_t)d.mp);
        const uint32_t gbytes = (uint32_t)d.db * 4u;  // bytes of one 4-row group of the direction map
        const __amdgpu_buffer_rsrc_t rdir = make_rsrc(d.dirs, (uint32_t)((H + 3) >> 2) * gbytes);
        const int P = (H + K - 1) / K;
        int w = W, k = 0;
#pragma unroll 1
        while (k < d.max_seams && w > 1 && sm.left > 0) {
            const unsigned long long tm0 = t == 0 ? wall_clock64() : 0ull;
            const bool act = j0 < w;
            const uint32_t v0 = act ? (uint32_t)(j0 * C) : kBufDrop;
            const uint32_t vl = act && j0 > 0 ? (uint32_t)(j0 * C - 4) : kBufDrop;
            const uint32_t mo = act ? (uint32_t)j0 : kBufDrop;
            const bool anc_in_lds = P * w <= ANC_LDS;
            uint8_t* const ancg = reinterpret_cast<uint8_t*>(d.anc);
            bool okR[CPL];  // column j0+c has a right neighbour
#pragma unroll
            for (int c = 0; c < CPL; ++c) okR[c] = j0 + c + 1 < w;

            // ---- DP over the rows with the masked e1 energy (64-bit keys)
            uint32_t Qh[CPL], Ql[CPL];  // key of each column: unmasked count; E << 9 | ancestor offset
            if (wv * 64 * CPL >= w) {
#pragma unroll 1
                for (int i = 1; i < H; ++i) lds_barrier();
            } else {
                uint32_t ring[PF][NDW], mring[PF][MD];
                static_for<PF>([&](auto U) {
                    constexpr int u = decltype(U)::value;
                    const uint32_t so = (uint32_t)min(u, H - 1);
                    load_row(ring[u], rwk, vl, v0, so * (uint32_t)d.wp);
                    load_mask(mring[u], rmk, mo, so * (uint32_t)d.mp);
                });
                uint32_t Pc[CPL + 2], Pu[CPL], dacc[CPL / 4];
                pixels(ring[0], Pc);
                if (t == 0) Pc[0] = Pc[1];  // left neighbour of column 0 clamped to it
#pragma unroll
                for (int c = 0; c < CPL; ++c) Pu[c] = Pc[c + 1];  // the row above row 0 is row 0
#pragma unroll
                for (int q = 0; q < CPL / 4; ++q) dacc[q] = 0;
                int kleft = K, phase = 0;
                auto row = [&](auto U, int i, auto LAST) {
                    constexpr int u = decltype(U)::value;
                    constexpr bool last = decltype(LAST)::value;  // the block holds row H-1: no refill
                    // the row below (clamped: the last row is its own lower neighbour)
                    uint32_t Pn[CPL + 2];
                    pixels(ring[(u + 1) % PF], Pn);
                    if (t == 0) Pn[0] = Pn[1];
                    if (last && i == H - 1) {
#pragma unroll
                        for (int c = 0; c < CPL + 2; ++c) Pn[c] = Pc[c];
                    }
                    uint32_t mw[MD];
#pragma unroll
                    for (int q = 0; q < MD; ++q) mw[q] = mring[u][q];
                    if (!last) {
                        const uint32_t so = (uint32_t)min(i + PF, H - 1);
                        load_row(ring[u], rwk, vl, v0, so * (uint32_t)d.wp);
                        load_mask(mring[u], rmk, mo, so * (uint32_t)d.mp);
                    }
                    uint32_t e[CPL], um[CPL];
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const uint32_t pr = okR[c] ? Pc[c + 2] : Pc[c + 1];
                        e[c] = __builtin_amdgcn_sad_u8(Pu[c], Pn[c + 1], __builtin_amdgcn_sad_u8(Pc[c], pr, 0u));
                        um[c] = ((mw[c >> 2] >> (8 * (c & 3))) & 0xFFu) == 0u ? 1u : 0u;
                    }
                    uint32_t bits = 0;
                    if (u == 0 && i == 0) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            Qh[c] = um[c];
                            Ql[c] = (e[c] << 9) | 64u;
                            bits |= 1u << (2 * c);
                        }
                    } else {
                        const int b = i & 1;
                        sm.xa[b][t] = ((unsigned long long)Qh[0] << 32) | Ql[0];
                        sm.xb[b][t + 1] = ((unsigned long long)Qh[CPL - 1] << 32) | Ql[CPL - 1];
                        lds_barrier();
                        const unsigned long long Kl = sm.xb[b][t], Kr = sm.xa[b][t + 1];
                        uint32_t Nh[CPL], Nl[CPL];
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            unsigned long long kL =
                                c == 0 ? Kl : (((unsigned long long)Qh[c - 1] << 32) | Ql[c - 1]);
                            if (c == 0 && t == 0) kL = INF;  // column 0 has no upper-left parent
                            const unsigned long long kU = ((unsigned long long)Qh[c] << 32) | (Ql[c] | 0x80u);
                            unsigned long long kR = INF;
                            if (okR[c])
                                kR = (c == CPL - 1 ? Kr : (((unsigned long long)Qh[c + 1] << 32) | Ql[c + 1])) | 0x100u;
                            const unsigned long long kk = min64(min64(kL, kU), kR);
                            Nl[c] = next_state((uint32_t)kk, e[c]);
                            Nh[c] = (uint32_t)(kk >> 32) + um[c];
                            bits |= (((uint32_t)kk >> 7) & 3u) << (2 * c);
                        }
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            Qh[c] = Nh[c];
                            Ql[c] = Nl[c];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < CPL; ++c) Pu[c] = Pc[c + 1];
#pragma unroll
                    for (int c = 0; c < CPL + 2; ++c) Pc[c] = Pn[c];
#pragma unroll
                    for (int q = 0; q < CPL / 4; ++q) dacc[q] |= ((bits >> (8 * q)) & 0xFFu) << (8 * (u & 3));
                    if ((u & 3) == 3 || (last && i == H - 1)) {
#pragma unroll
                        for (int q = 0; q < CPL / 4; ++q) {
                            const uint32_t vo = j0 + 4 * q < w ? (uint32_t)(j0 / 4 + q) * 4u : kBufDrop;
                            __builtin_amdgcn_raw_buffer_store_b32(dacc[q], rdir, (int)vo,
                                                                  (int)((uint32_t)(i >> 2) * gbytes), 0);
                            dacc[q] = 0;
                        }
                    }
                    if (--kleft == 0 || (last && i == H - 1)) {
                        // end of a phase: record the ancestor offsets, then restart them
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            if (j0 + c < w) {
                                if (anc_in_lds) anc_lds[phase * w + j0 + c] = (uint8_t)(Ql[c] & 0x7Fu);
                                else *gp(ancg + phase * w + j0 + c) = (uint8_t)(Ql[c] & 0x7Fu);
                            }
                            Ql[c] = (Ql[c] & ~0x7Fu) | 64u;
                        }
                        kleft = K;
                        ++phase;
                    }
                };
                int i0 = 0;
#pragma unroll 1
                for (; i0 + PF < H; i0 += PF)
                    static_for<PF>([&](auto U) { row(U, i0 + decltype(U)::value, std::false_type{}); });
                static_for<PF>([&](auto U) {
                    if (i0 + decltype(U)::value < H) row(U, i0 + decltype(U)::value, std::true_type{});
                });
            }

            // ---- argmin of the last row: (q << 37 | E << 14 | column), the leftmost minimum
            unsigned long long best = INF;
            if (wv * 64 * CPL < w) {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (j0 + c < w)
                        best = min64(best, ((unsigned long long)Qh[c] << 37) |
                                               ((unsigned long long)(Ql[c] >> 9) << 14) | (unsigned)(j0 + c));
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) best = min64(best, (unsigned long long)__shfl_xor((long long)best, o));
            if (lane == 0) sm.red[wv] = best;
            __syncthreads();
            const unsigned long long tm1 = t == 0 ? wall_clock64() : 0ull;
            if (t == 0) {
                unsigned long long b = sm.red[0];
                for (int x = 1; x < NW; ++x) b = min64(b, sm.red[x]);
                int je = (int)(b & 0x3FFFull);
                const long long q = (long long)(b >> 37), E = (long long)((b >> 14) & 0x7FFFFFull);
                const long long m = (long long)H - q;  // masked pixels on the seam
                if (d.costs_out) d.costs_out[k] = E - bias * m;
                sm.left -= (int)m;
                // ---- backtrack, first hop: phase by phase through the ancestor offsets
                sm.jend[P - 1] = je;
                for (int p = P - 1; p > 0; --p) {
                    const int a = anc_in_lds ? (int)anc_lds[p * w + je] : (int)*gp(ancg + p * w + je);
                    je = min(max(je + a - 64, 0), w - 1);
                    sm.jend[p - 1] = je;
                }
            }
            __syncthreads();
            // ---- then every phase's rows, one wave per phase, from an LDS window of the map
#pragma unroll 1
            for (int p = wv; p < P; p += NW) {
                const int r0 = p * K, n = min(K, H - r0), ng = (n + 3) >> 2;
                const int je = sm.jend[p];
                const int cb0 = max(0, je - (K - 1)) >> 2;
                uint32_t* win = sm.win[wv];
                constexpr int NI = (GK * WD + 63) / 64;
                uint32_t v[NI];
                const uint32_t* src = reinterpret_cast<const uint32_t*>(d.dirs) + (size_t)(r0 >> 2) * d.db;
#pragma unroll
                for (int mi = 0; mi < NI; ++mi) {
                    const int x = lane + 64 * mi, g = x / WD, qd = x % WD;
                    v[mi] = g < ng && cb0 + qd < d.db ? *gp(src + (size_t)g * d.db + cb0 + qd) : 0u;
                }
#pragma unroll
                for (int mi = 0; mi < NI; ++mi) {
                    const int x = lane + 64 * mi;
                    if (x < GK * WD) win[x] = v[mi];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int s = je, mys = 0;
                for (int i = n - 1; i >= 0; --i) {
                    if (lane == i) mys = s;
                    if (i > 0) {
                        const int qd = min(max((s >> 2) - cb0, 0), WD - 1);
                        const uint32_t wd = win[(i >> 2) * WD + qd];
                        s += (int)((wd >> ((i & 3) * 8 + (s & 3) * 2)) & 3u) - 1;
                        s = min(max(s, 0), w - 1);
                    }
                }
                if (lane < n) {
                    *gp(d.seam + r0 + lane) = mys;
                    if (d.seams_out) *gp(d.seams_out + (size_t)k * H + r0 + lane) = mys;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            __syncthreads();
            const unsigned long long tm2 = t == 0 ? wall_clock64() : 0ull;
            // ---- removal: in each seam row the pixels and the mask bytes right of the seam move one
            // column left; two rows (pixel and mask segments of each) per memory round trip, the
            // 2-row groups dealt to the waves round-robin
#pragma unroll 1
            for (int r0 = wv * 2; r0 < H; r0 += NW * 2) {
                const int n = min(2, H - r0);
                const int sv = lane < n ? *gp(d.seam + r0 + lane) : 0;
                auto segs = [&](int i, SSeg& gi, SSeg& gm) {
                    if (i >= n) {
                        gi.base = gm.base = d.wk;
                        gi.q0 = gi.q1 = gi.sh = gi.n = 0;
                        gm.q0 = gm.q1 = gm.sh = gm.n = 0;
                        return;
                    }
                    const int si = min(max(__builtin_amdgcn_readlane(sv, i), 0), w - 1);
                    uint8_t* r = d.wk + (long long)(r0 + i) * d.wp;
                    uint8_t* mr = d.mk + (long long)(r0 + i) * d.mp;
                    gi = sseg<false>(r + (long long)si * C, r + (long long)(w - 1) * C, C);
                    gm = sseg<false>(mr + si, mr + (w - 1), 1);
                };
                SSeg a0, a1, b0, b1;
                segs(0, a0, a1);
                segs(1, b0, b1);
                shift_rows2_wave<1, false, false>(a0, a1, b0, b1, lane);
            }
            __syncthreads();
            if (t == 0) {  // device clock per stage: DP sweep; argmin + backtrack; removal
                const unsigned long long tm3 = wall_clock64();
                ctl->t_stage[0] += tm1 - tm0;
                ctl->t_stage[1] += tm2 - tm1;
                ctl->t_stage[2] += tm3 - tm2;
            }
            ++k;
            --w;
        }
        // ---- the carved rows go from wk to out (when the caller wants them there)
        if (d.out && k > 0) {
            const int nb = w * C;
#pragma unroll 1
            for (int r = wv; r < H; r += NW)
                copy_bytes_wave(d.out + (long long)r * d.out_pitch, d.wk + (long long)r * d.wp, nb, lane);
        }
        __syncthreads();
        if (t == 0) {
            ctl->k = k;
            ctl->left = sm.left;
            ctl->w = w;
            ctl->t_end = wall_clock64();
        }
    }
};

}  // namespace obj

// One workgroup per image of `imgs`.
template <int CPL>
__global__ __launch_bounds__(obj::NT, 1) void obj_carve_kernel(const ObjImg* __restrict__ imgs, int n) {
    __shared__ obj::Smem sm;
    __shared__ uint8_t anc[obj::ANC_LDS];
    if ((int)blockIdx.x >= n) return;
    const ObjImg d = imgs[blockIdx.x];
    switch (d.C) {
        case 1: obj::Carver<1, CPL>::carve(d, sm, anc); break;
        case 2: obj::Carver<2, CPL>::carve(d, sm, anc); break;
        case 3: obj::Carver<3, CPL>::carve(d, sm, anc); break;
        default: obj::Carver<4, CPL>::carve(d, sm, anc); break;
    }
}

// Zero the control words of n images (the carve accumulates its stage clocks into them) and set
// the mask bounding box to empty.
__global__ void obj_reset_kernel(ObjCtl* ctl, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ObjCtl* c = ctl + i;
    c->k = c->left = c->w = 0;
    c->bbox[0] = c->bbox[2] = 0x7FFFFFFF;
    c->bbox[1] = c->bbox[3] = -1;
    c->t_begin = c->t_end = 0;
    c->t_stage[0] = c->t_stage[1] = c->t_stage[2] = 0;
}

// Bounding box of the nonzero bytes of an H x W mask: bbox = {first row, last row, first
// column, last column} (atomic min / max over the rows; bbox starts as {max, -1, max, -1}).
__global__ void mask_bbox_kernel(const uint8_t* __restrict__ mask, int H, int W, long long mpitch, int* bbox) {
    const int y = blockIdx.x;
    if (y >= H) return;
    const uint8_t* r = mask + (long long)y * mpitch;
    int c0 = 0x7FFFFFFF, c1 = -1;
    for (int x = threadIdx.x; x < W; x += blockDim.x)
        if (*gp(r + x)) {
            c0 = min(c0, x);
            c1 = max(c1, x);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c0 = min(c0, __shfl_xor(c0, o));
        c1 = max(c1, __shfl_xor(c1, o));
    }
    if ((threadIdx.x & 63) == 0 && c1 >= 0) {
        atomicMin(bbox + 0, y);
        atomicMax(bbox + 1, y);
        atomicMin(bbox + 2, c0);
        atomicMax(bbox + 3, c1);
    }
}

// dst rows take `bytes` bytes of the src rows, one wave per row.
__global__ void copy_rows_kernel(const uint8_t* __restrict__ src, long long sp, uint8_t* __restrict__ dst,
                                 long long dp, int rows, int bytes) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int r = wv; r < rows; r += nw) copy_bytes_wave(dst + (long long)r * dp, src + (long long)r * sp, bytes, lane);
}

hipError_t launch_obj_reset(ObjCtl* ctl, int n, hipStream_t st) {
    hipLaunchKernelGGL(obj_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ctl, n);
    return hipGetLastError();
}

hipError_t launch_obj_carve(const ObjImg* imgs, int n, int max_w, hipStream_t st) {
    if (max_w > kFwdMaxW) return hipErrorInvalidValue;
    if (max_w <= 4096) hipLaunchKernelGGL(obj_carve_kernel<4>, dim3(n), dim3(obj::NT), 0, st, imgs, n);
    else hipLaunchKernelGGL(obj_carve_kernel<8>, dim3(n), dim3(obj::NT), 0, st, imgs, n);
    return hipGetLastError();
}

hipError_t launch_mask_bbox(const uint8_t* mask, int H, int W, long long mpitch, int* bbox, hipStream_t st) {
    hipLaunchKernelGGL(mask_bbox_kernel, dim3(H), dim3(256), 0, st, mask, H, W, mpitch, bbox);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const uint8_t* src, long long sp, uint8_t* dst, long long dp, int rows, int bytes,
                            hipStream_t st) {
    const int waves = rows < 4096 ? rows : 4096;
    hipLaunchKernelGGL(copy_rows_kernel, dim3((waves + 3) / 4), dim3(256), 0, st, src, sp, dst, dp, rows, bytes);
    return hipGetLastError();
}

}  // namespace sc
