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
//    shifted into a byte per lane with v_alignbit and stored as a 2-bit map.
//  * A wave owns a strip of S = 64*CPL - 2*KR columns and computes KR halo
//    columns on each side, so it runs KR rows with no exchange at all
//    ("ghost zone" tiling); waves exchange the last row of every KR-row phase
//    through memory and a barrier.
//  * At the last row of each phase every owned column records how far its
//    minimal path moved within the phase; the backtrack then hops phase by
//    phase (one load per phase) and walks the KR rows of every phase in
//    parallel from an LDS window of the direction map.
//  * Removal shifts the bytes right of the seam one pixel left, row-parallel
//    with coalesced 16-byte slots, for the image and the energy plane alike;
//    the energy is then recomputed only at the two new columns {s-1, s} of
//    each row (the only cells whose stencil changed).
#include <type_traits>

#include "sc_internal.h"

namespace sc {

constexpr uint32_t QINF = 0xFFFFFF00u;  // "+infinity" key: larger than any real key, +10 cannot wrap
constexpr unsigned kStatusTimeout = 1u;

// ----------------------------------------------------------------------------------------------
// e1 energy at one pixel of the current image (width w), indices clamped to the image.
__device__ __forceinline__ uint32_t energy_at(const uint8_t* __restrict__ img, long long pitch, int H, int w,
                                              int C, int y, int x) {
    const int xl = x > 0 ? x - 1 : 0, xr = x + 1 < w ? x + 1 : w - 1;
    const int yu = y > 0 ? y - 1 : 0, yd = y + 1 < H ? y + 1 : H - 1;
    const uint8_t* r = img + (long long)y * pitch;
    const uint8_t* ru = img + (long long)yu * pitch;
    const uint8_t* rd = img + (long long)yd * pitch;
    uint32_t s = 0;
    for (int c = 0; c < C; ++c) {
        const int dx = (int)r[xr * C + c] - (int)r[xl * C + c];
        const int dy = (int)rd[x * C + c] - (int)ru[x * C + c];
        s += (uint32_t)(dx < 0 ? -dx : dx) + (uint32_t)(dy < 0 ? -dy : dy);
    }
    return s;
}

// Standalone energy map (int32, dense).
__global__ void energy_i32_kernel(const uint8_t* __restrict__ img, int H, int W, int C, long long pitch,
                                  int32_t* __restrict__ out) {
    const int y = blockIdx.y;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < W; x += gridDim.x * blockDim.x)
        out[(long long)y * W + x] = (int32_t)energy_at(img, pitch, H, W, C, y, x);
}

// Per-image preparation: zero the control words, optionally copy src -> img, fill the energy plane.
__device__ void prepare_rows(const Img& d, int row_begin, int row_step) {
    const uint8_t* srcimg = d.src ? d.src : d.img;
    if (row_begin == 0 && threadIdx.x == 0) {
        Ctl* c = reinterpret_cast<Ctl*>(d.amin);
        c->amin = ~0ull;
        c->bar = 0;
        c->status = 0;
        c->t_begin = c->t_end = 0;
    }
    for (int y = row_begin; y < d.H; y += row_step) {
        uint16_t* er = d.e + (long long)y * d.ep;
        for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
            er[x] = (uint16_t)energy_at(srcimg, d.pitch, d.H, d.W, d.C, y, x);
            if (d.src) {
                const uint8_t* s = d.src + (long long)y * d.pitch + (long long)x * d.C;
                uint8_t* o = d.img + (long long)y * d.pitch + (long long)x * d.C;
                for (int c = 0; c < d.C; ++c) o[c] = s[c];
            }
        }
    }
}

// A single-image workspace starts with a header just before its one Ctl block.
__device__ __forceinline__ void write_single_header(const Img& d) {
    uint32_t* h = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d.amin) - kWsHeadBytes);
    h[0] = kWsMagic;
    h[1] = 1u;
}

__global__ void prepare_single_kernel(Img d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) write_single_header(d);
    prepare_rows(d, blockIdx.x, gridDim.x);
}

__global__ void prepare_batch_kernel(const Img* __restrict__ imgs, int n) {
    const int i = blockIdx.y;
    if (i < n) {
        Img d = imgs[i];
        prepare_rows(d, blockIdx.x, gridDim.x);
    }
}

// Energy plane from a caller's int32 energy map (sc_dp_seam).
__global__ void prepare_from_i32_kernel(Img d, const int32_t* __restrict__ e) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        write_single_header(d);
        Ctl* c = reinterpret_cast<Ctl*>(d.amin);
        c->amin = ~0ull;
        c->bar = 0;
        c->status = 0;
    }
    const int y = blockIdx.y;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < d.W; x += gridDim.x * blockDim.x)
        d.e[(long long)y * d.ep + x] = (uint16_t)e[(long long)y * d.W + x];
}

// ----------------------------------------------------------------------------------------------
// In-place left shift of one row segment by `sh` bytes (1 <= sh <= 4), one wave:
// dst byte x gets src byte x+sh for x in [lo, hi) (addresses).  Work is cut into
// 16-byte slots aligned to absolute addresses; each lane owns one slot per pass.
// All loads of a pass are issued before its stores and a pass only reads slots at
// or after its own, so the in-place update is hazard free.
template <int U>
__device__ __forceinline__ void shift_left_wave(uint8_t* lo_p, uint8_t* hi_p, int sh, int lane) {
    const uintptr_t lo = (uintptr_t)lo_p, hi = (uintptr_t)hi_p;
    if (lo >= hi) return;
    const uintptr_t q0 = lo >> 4, q1 = (hi - 1) >> 4;
    // every address is formed from lo_p so the compiler keeps the global address space
    uint8_t* const base = lo_p - (lo & 15);  // = (q0 << 4)
    for (uintptr_t qb = q0; qb <= q1; qb += 64 * U) {
        uint4 A[U];
        uint32_t B[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uintptr_t q = qb + (uintptr_t)(u * 64 + lane);
            A[u] = make_uint4(0, 0, 0, 0);
            B[u] = 0;
            if (q <= q1) {
                const uint8_t* sp = base + ((q - q0) << 4);
                A[u] = *reinterpret_cast<const uint4*>(sp);
                if ((q << 4) + 16 - sh < hi) B[u] = *reinterpret_cast<const uint32_t*>(sp + 16);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uintptr_t q = qb + (uintptr_t)(u * 64 + lane);
            if (q > q1) continue;
            const uint32_t D[5] = {A[u].x, A[u].y, A[u].z, A[u].w, B[u]};
            uint32_t o[4];
            if (sh == 4) {
                o[0] = D[1]; o[1] = D[2]; o[2] = D[3]; o[3] = D[4];
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbyte(D[i + 1], D[i], (uint32_t)sh);
            }
            const uintptr_t s0 = q << 4;
            uint8_t* dp = base + ((q - q0) << 4);
            if (s0 >= lo && s0 + 16 <= hi) {
                *reinterpret_cast<uint4*>(dp) = make_uint4(o[0], o[1], o[2], o[3]);
            } else {
                const uint32_t k0 = s0 > lo ? 0u : (uint32_t)(lo - s0);
                const uint32_t k1 = s0 + 16 < hi ? 16u : (uint32_t)(hi - s0);
                for (uint32_t k = k0; k < k1; ++k) dp[k] = (uint8_t)(o[k >> 2] >> ((k & 3) * 8));
            }
        }
    }
}

// Standalone seam removal: one wave per row.
__global__ void remove_seam_kernel(uint8_t* __restrict__ img, int H, int W, int C, long long pitch,
                                   const int32_t* __restrict__ seam) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int y = wv; y < H; y += nw) {
        const int s = seam[y];
        if (s < 0 || s >= W) continue;
        uint8_t* row = img + (long long)y * pitch;
        shift_left_wave<4>(row + (long long)s * C, row + (long long)(W - 1) * C, C, lane);
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
            for (int c = 0; c < C; ++c) tile[r][tx * C + c] = src[(long long)y * sp + (long long)x * C + c];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int x = bx + r, y = by + tx;  // output row x, column y
        if (y < H && x < W)
            for (int c = 0; c < C; ++c) dst[(long long)x * dp + (long long)y * C + c] = tile[tx][r * C + c];
    }
}

// ----------------------------------------------------------------------------------------------
// Team barrier.  Within one workgroup a workgroup barrier suffices; workgroups of one team
// publish their writes with an agent-scope fence and meet at a counter in the image's
// control block.  The wait is bounded: after ~10 s it flags the image and gives up.
__device__ __forceinline__ bool team_sync(const Img& d, unsigned& epoch, int G, int* abort_flag) {
    if (G == 1) {
        __syncthreads();
        return true;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += (unsigned)G;
        __hip_atomic_fetch_add(d.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = wall_clock64();
        int ab = 0;
        while (__hip_atomic_load(d.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (__hip_atomic_load(d.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStatusTimeout) {
                ab = 1;
                break;
            }
            if (wall_clock64() - t0 > 1000000000ull) {  // 10 s at the 100 MHz constant clock
                __hip_atomic_fetch_or(d.status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
        }
        *abort_flag = ab;
    }
    __syncthreads();
    __threadfence();
    return *abort_flag == 0;
}

// ----------------------------------------------------------------------------------------------
// The carve engine: one image, carved by a team of G workgroups of NT threads.
template <int CPL, int KR, int NT>
struct Carver {
    static constexpr int WIN = 64 * CPL;       // columns a wave computes
    static constexpr int S = WIN - 2 * KR;     // columns a wave owns
    static constexpr int NW = NT / 64;         // waves per workgroup
    static constexpr int PF = 8;               // rows of energy prefetched ahead
    static constexpr int WD = (KR / 2 + 2 + 3) / 4 + 1;  // dwords of a backtrack window row
    static constexpr int PMAX = 16448 / KR + 2;          // phases of the tallest image
    static_assert(CPL == 4 || CPL == 8, "a lane's directions fill a byte or a short");
    static_assert(KR % CPL == 0 && KR <= 63 && S > 0 && S % 16 == 0, "phase shape");

    struct Smem {
        int jend[PMAX];            // seam column at the last row of every phase
        uint32_t win[NW][KR * WD]; // backtrack windows of the direction map
        int abort_flag;
    };

    using EV = typename std::conditional<CPL == 4, uint2, uint4>::type;

    static __device__ __forceinline__ void unpack(const EV& v, uint32_t (&e)[CPL]) {
        if constexpr (CPL == 4) {
            e[0] = v.x & 0xffffu; e[1] = v.x >> 16; e[2] = v.y & 0xffffu; e[3] = v.y >> 16;
        } else {
            e[0] = v.x & 0xffffu; e[1] = v.x >> 16; e[2] = v.y & 0xffffu; e[3] = v.y >> 16;
            e[4] = v.z & 0xffffu; e[5] = v.z >> 16; e[6] = v.w & 0xffffu; e[7] = v.w >> 16;
        }
    }

    // One DP row for the CPL columns of this lane.  Q holds the previous row's keys (tags in
    // bits [1:0] are ignored); on return it holds this row's keys and `acc` the new directions
    // in its top 2*CPL bits (column 0 lowest).
    static __device__ __forceinline__ uint32_t row_step(uint32_t (&Q)[CPL], const uint32_t (&e)[CPL]) {
        uint32_t t[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) t[k] = Q[k] & ~3u;
        // left neighbour of column 0 lives in lane-1, right neighbour of the last column in lane+1
        const uint32_t left = (uint32_t)__builtin_amdgcn_update_dpp((int)QINF, (int)t[CPL - 1], 0x138, 0xf, 0xf, false);
        const uint32_t right = (uint32_t)__builtin_amdgcn_update_dpp((int)QINF, (int)t[0], 0x130, 0xf, 0xf, false);
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const uint32_t L = k ? t[k - 1] : left;                 // tag 0, offset +0
            const uint32_t Cc = t[k] + 5u;                          // tag 1, offset +1
            const uint32_t R = (k + 1 < CPL ? t[k + 1] : right) + 10u;  // tag 2, offset +2
            const uint32_t r = min(min(L, Cc), R);
            Q[k] = r + (e[k] << 9);
            acc = __builtin_amdgcn_alignbit(r, acc, 2u);
        }
        return acc;
    }

    // One strip (t) of one phase (rows r0..r1-1) for the calling wave.
    template <bool EDGE>
    static __device__ void dp_item(const Img& d, int w, int p, int r0, int r1, int t, int lane) {
        const int base = t * S - KR;
        const int col0 = base + lane * CPL;
        const bool lane_any = col0 >= 0 && col0 < w;
        const bool owned = lane >= KR / CPL && lane < (KR + S) / CPL && col0 < w;
        bool valid[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) valid[k] = (col0 + k >= 0) && (col0 + k < w);

        uint32_t Q[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) Q[k] = QINF;
        if (p > 0 && lane_any) {
            const uint32_t* xr = d.xq + (size_t)((p - 1) & 1) * d.xw + col0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) Q[k] = valid[k] ? (xr[k] & ~0x1FFu) : QINF;  // offset and tag reset
        }

        const uint16_t* erow = d.e + (size_t)r0 * d.ep + (lane_any ? col0 : 0);
        EV ring[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            ring[i] = EV{};
            if (r0 + i < r1 && lane_any) ring[i] = *reinterpret_cast<const EV*>(erow + (size_t)i * d.ep);
        }
        uint8_t* drow = d.dirs + (size_t)r0 * d.db + (col0 >> 2);
        for (int rb = r0; rb < r1; rb += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                const int r = rb + i;
                if (r < r1) {
                    const EV ev = ring[i];
                    if (r + PF < r1 && lane_any)
                        ring[i] = *reinterpret_cast<const EV*>(erow + (size_t)(r - r0 + PF) * d.ep);
                    uint32_t e[CPL];
                    unpack(ev, e);
                    if (r == 0) {
#pragma unroll
                        for (int k = 0; k < CPL; ++k) Q[k] = valid[k] ? (e[k] << 9) : QINF;
                    } else {
                        const uint32_t acc = row_step(Q, e);
                        if (EDGE) {
#pragma unroll
                            for (int k = 0; k < CPL; ++k) Q[k] = valid[k] ? Q[k] : QINF;
                        }
                        if (owned) {
                            uint8_t* dp = drow + (size_t)(r - r0) * d.db;
                            if constexpr (CPL == 4) *dp = (uint8_t)(acc >> 24);
                            else *reinterpret_cast<uint16_t*>(dp) = (uint16_t)(acc >> 16);
                        }
                    }
                }
            }
        }
        // phase end: publish the last row of the owned columns and the ancestor offsets
        if (owned) {
            uint32_t* xw = d.xq + (size_t)(p & 1) * d.xw + col0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) xw[k] = Q[k];
            if (p > 0) {
                const int n = r1 - r0;
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if (valid[k]) d.anc[(size_t)p * d.W + col0 + k] = (int8_t)((int)((Q[k] >> 2) & 127u) - n);
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
            if (lane == 0 && key != ~0ull) atomicMin(d.amin, key);
        }
    }

    static __device__ void carve_image(const Img& d, int rank, int G, Smem& sm) {
        Ctl* ctl = reinterpret_cast<Ctl*>(d.amin);
        if (rank == 0 && threadIdx.x == 0) ctl->t_begin = wall_clock64();
        carve_seams(d, rank, G, sm);
        __syncthreads();
        if (rank == 0 && threadIdx.x == 0) ctl->t_end = wall_clock64();
    }

    static __device__ void carve_seams(const Img& d, int rank, int G, Smem& sm) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int TW = G * NW, tw = rank * NW + wv;
        const int H = d.H, P = d.P;
        unsigned epoch = 0;
        const int nseams = d.mode ? 1 : d.W - d.target_w;
        int w = d.W;
        for (int k = 0; k < nseams; ++k, --w) {
            // ---- DP sweep, phase by phase (a3) and the bottom-row argmin (a4)
            const int nstr = (w + S - 1) / S;
            for (int p = 0; p < P; ++p) {
                const int r0 = p * KR, r1 = min(H, r0 + KR);
                for (int t = tw; t < nstr; t += TW) {
                    const int base = t * S - KR;
                    if (base < 0 || base + WIN > w) dp_item<true>(d, w, p, r0, r1, t, lane);
                    else dp_item<false>(d, w, p, r0, r1, t, lane);
                }
                if (!team_sync(d, epoch, G, &sm.abort_flag)) return;
            }
            const unsigned long long key =
                __hip_atomic_load(d.amin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int jstar = (int)(key & 0xffffffffu);
            if (rank == 0 && threadIdx.x == 0 && d.costs_out) d.costs_out[k] = (long long)(key >> 32);
            // ---- backtrack (a5): hop phase ends, then walk every phase's rows in parallel
            if (threadIdx.x == 0) {
                // every column is clamped into [0, w) before it indexes memory
                int j = min(max(jstar, 0), w - 1);
                sm.jend[P - 1] = j;
                for (int p = P - 1; p >= 1; --p) {
                    j = min(max(j + d.anc[(size_t)p * d.W + j], 0), w - 1);
                    sm.jend[p - 1] = j;
                }
            }
            __syncthreads();
            for (int p = tw; p < P; p += TW) {
                const int r0 = p * KR, r1 = min(H, r0 + KR), n = r1 - r0;
                const int je = sm.jend[p];
                const int dlo = (max(0, je - KR) >> 2) >> 2;
                const int ndw = d.db >> 2;
                uint32_t* win = sm.win[wv];
                if (lane < n) {
                    const uint32_t* src = reinterpret_cast<const uint32_t*>(d.dirs + (size_t)(r0 + lane) * d.db);
#pragma unroll
                    for (int q = 0; q < WD; ++q) win[lane * WD + q] = (dlo + q < ndw) ? src[dlo + q] : 0u;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int s = je, mys = 0;
                for (int i = n - 1; i >= 0; --i) {
                    if (lane == i) mys = s;
                    if (i > 0) {
                        const int b = s >> 2;
                        const int q = min(max((b >> 2) - dlo, 0), WD - 1);
                        const uint32_t wd = win[i * WD + q];
                        s += (int)((wd >> ((b & 3) * 8 + (s & 3) * 2)) & 3u) - 1;
                        s = min(max(s, 0), w - 1);
                    }
                }
                if (lane < n) {
                    d.seam[r0 + lane] = mys;
                    if (d.seams_out) d.seams_out[(size_t)k * H + r0 + lane] = mys;
                }
                __builtin_amdgcn_wave_barrier();
                if (!d.mode) {
                    // ---- removal (a6) of this phase's rows: image bytes and energy plane
                    for (int i = 0; i < n; ++i) {
                        const int si = __shfl(mys, i, 64);
                        uint8_t* row = d.img + (long long)(r0 + i) * d.pitch;
                        shift_left_wave<4>(row + (long long)si * d.C, row + (long long)(w - 1) * d.C, d.C, lane);
                        uint8_t* er = reinterpret_cast<uint8_t*>(d.e + (size_t)(r0 + i) * d.ep);
                        shift_left_wave<2>(er + 2 * si, er + 2 * (w - 1), 2, lane);
                    }
                }
            }
            if (!team_sync(d, epoch, G, &sm.abort_flag)) return;
            if (d.mode) break;
            if (rank == 0 && threadIdx.x == 0)
                __hip_atomic_store(d.amin, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // ---- band energy (a2): only new columns s-1 and s of each row changed
            const int w2 = w - 1;
            for (int r = tw * 64 + lane; r < H; r += TW * 64) {
                const int s = min(max(d.seam[r], 0), w - 1);
                uint16_t* er = d.e + (size_t)r * d.ep;
                if (s - 1 >= 0 && s - 1 < w2) er[s - 1] = (uint16_t)energy_at(d.img, d.pitch, H, w2, d.C, r, s - 1);
                if (s < w2) er[s] = (uint16_t)energy_at(d.img, d.pitch, H, w2, d.C, r, s);
            }
            if (!team_sync(d, epoch, G, &sm.abort_flag)) return;
        }
    }
};

template <int CPL, int KR, int NT>
__global__ __launch_bounds__(NT) void carve_single_kernel(Img d) {
    using CV = Carver<CPL, KR, NT>;
    __shared__ typename CV::Smem sm;
    // Team members are blocks 0, 8, 16, ... so that they share one XCD's L2 under the
    // round-robin dispatch of workgroups to XCDs; the other blocks exit at once.
    if (blockIdx.x & 7) return;
    CV::carve_image(d, blockIdx.x >> 3, d.G, sm);
}

// Batched carve: block b is member blk[b].y of team blk[b].x; team t carves the images
// team_imgs[teams[t].x .. teams[t].x + teams[t].y) one after another.
template <int CPL, int KR, int NT>
__global__ __launch_bounds__(NT) void carve_batch_kernel(const Img* __restrict__ imgs, const int2* __restrict__ blk,
                                                         const int2* __restrict__ teams,
                                                         const int* __restrict__ team_imgs) {
    using CV = Carver<CPL, KR, NT>;
    __shared__ typename CV::Smem sm;
    const int2 me = blk[blockIdx.x];
    if (me.x < 0) return;
    const int2 tr = teams[me.x];
    for (int i = 0; i < tr.y; ++i) {
        const Img d = imgs[team_imgs[tr.x + i]];
        CV::carve_image(d, me.y, d.G, sm);
        __syncthreads();
    }
}

// Unpack the 2-bit direction map into bytes (row 0 has no parent: 1).
__global__ void unpack_dirs_kernel(Img d, uint8_t* __restrict__ out) {
    const int y = blockIdx.y;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < d.W; x += gridDim.x * blockDim.x) {
        uint8_t v = 1;
        if (y > 0) v = (d.dirs[(size_t)y * d.db + (x >> 2)] >> ((x & 3) * 2)) & 3u;
        out[(size_t)y * d.W + x] = v;
    }
}

// ----------------------------------------------------------------------------------------------
// Variant table and launchers.
static const Variant kVariants[] = {
    {4, 32, 256, "cpl4_k32_t256"},
    {4, 32, 512, "cpl4_k32_t512"},
    {4, 32, 1024, "cpl4_k32_t1024"},
    {8, 48, 256, "cpl8_k48_t256"},
    {8, 48, 1024, "cpl8_k48_t1024"},
};
int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const Variant& variant(int v) { return kVariants[v]; }
int default_variant() { return 2; }
int max_phase_rows() { return 48; }

template <int CPL, int KR, int NT>
static hipError_t launch_single_t(const Img& d, int G, hipStream_t st) {
    hipLaunchKernelGGL((carve_single_kernel<CPL, KR, NT>), dim3(8 * G), dim3(NT), 0, st, d);
    return hipGetLastError();
}

template <int CPL, int KR, int NT>
static hipError_t launch_batch_t(const Img* imgs, const int2* blk, const int2* teams, const int* ti, int nb,
                                 hipStream_t st) {
    hipLaunchKernelGGL((carve_batch_kernel<CPL, KR, NT>), dim3(nb), dim3(NT), 0, st, imgs, blk, teams, ti);
    return hipGetLastError();
}

template <int CPL, int KR, int NT>
static int occupancy_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, carve_batch_kernel<CPL, KR, NT>, NT, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_carve_single(const Img& d, int v, int G, hipStream_t st) {
    switch (v) {
        case 0: return launch_single_t<4, 32, 256>(d, G, st);
        case 1: return launch_single_t<4, 32, 512>(d, G, st);
        case 2: return launch_single_t<4, 32, 1024>(d, G, st);
        case 3: return launch_single_t<8, 48, 256>(d, G, st);
        case 4: return launch_single_t<8, 48, 1024>(d, G, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_carve_batch(const Img* imgs, const int2* blk, const int2* teams, const int* ti, int nb, int v,
                              hipStream_t st) {
    switch (v) {
        case 0: return launch_batch_t<4, 32, 256>(imgs, blk, teams, ti, nb, st);
        case 1: return launch_batch_t<4, 32, 512>(imgs, blk, teams, ti, nb, st);
        case 2: return launch_batch_t<4, 32, 1024>(imgs, blk, teams, ti, nb, st);
        case 3: return launch_batch_t<8, 48, 256>(imgs, blk, teams, ti, nb, st);
        case 4: return launch_batch_t<8, 48, 1024>(imgs, blk, teams, ti, nb, st);
        default: return hipErrorInvalidValue;
    }
}

int carve_blocks_per_cu(int v) {
    switch (v) {
        case 0: return occupancy_t<4, 32, 256>();
        case 1: return occupancy_t<4, 32, 512>();
        case 2: return occupancy_t<4, 32, 1024>();
        case 3: return occupancy_t<8, 48, 256>();
        case 4: return occupancy_t<8, 48, 1024>();
        default: return 0;
    }
}

hipError_t launch_energy_i32(const uint8_t* img, int H, int W, int C, long long pitch, int32_t* out, hipStream_t st) {
    dim3 grid((W + 255) / 256, H);
    hipLaunchKernelGGL(energy_i32_kernel, grid, dim3(256), 0, st, img, H, W, C, pitch, out);
    return hipGetLastError();
}

hipError_t launch_prepare_single(const Img& d, hipStream_t st) {
    const int blocks = d.H < 2048 ? d.H : 2048;
    hipLaunchKernelGGL(prepare_single_kernel, dim3(blocks), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_prepare_from_i32(const Img& d, const int32_t* e, hipStream_t st) {
    dim3 grid((d.W + 255) / 256, d.H);
    hipLaunchKernelGGL(prepare_from_i32_kernel, grid, dim3(256), 0, st, d, e);
    return hipGetLastError();
}

hipError_t launch_prepare_batch(const Img* imgs, int n, int max_rows, hipStream_t st) {
    const int per = max_rows < 64 ? max_rows : 64;
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

}  // namespace sc
