// Forward-energy carve by teams of workgroups (sec. "Forward Energy Calculation", the standard
// definition with no per-pixel term; readings R17-R19): the DP cost of a pixel is the difference
// of the pixel pairs its removal makes neighbours, CU = D(left, right), plus D(up, left) for the
// upper-left parent or D(up, right) for the upper-right one, D = the channel sum of absolute
// differences (one v_sad_u8 on packed channels), neighbour indices clamped to the row.  The costs
// come from the current pixels, so there is no energy plane and no band update.
//
// Layout.  The working copy keeps one dword per pixel (channels in the low C bytes, zeros above),
// so a lane's 4 pixels are one 16-byte load and D is one v_sad_u8.
//
// Tiling.  A key is M << 9 | a, a = 64 + (ancestor column at the phase start) - (column), with
// the candidate's tag in bits 7-8 while the three parents are compared (ties to the leftmost
// parent, R5).  A wrong key at the edge of a tile moves one column inward per row, so a tile
// stays exact at distance n from its edges for n rows after its edges were last refreshed:
//  * a wave computes 256 columns (4 per lane; neighbours' keys and pixels by DPP wave shifts) and
//    its middle 240 (its core) are exact: every 8 rows the waves of a workgroup refresh the 8
//    columns on each side of their cores from their neighbours' cores through LDS;
//  * a workgroup computes the 976 columns of its 4 waves; in a team of several DP members, member
//    g computes [g*S - X, g*S + S + X) and owns [g*S, g*S + S), S = 976 - 2X, X = 2K = 112, and
//    at the end of every second phase of K = 56 rows it publishes its owned keys with the phase's
//    tag and reads the keys of its outer X columns on each side once they carry that tag (bounded
//    wait); an image of at most 968 columns has one DP member, whose columns from 0 are exact.
// A member takes part in a seam's DP only while some of its owned columns are in the image, so
// two neighbouring participants always wait for each other's keys at every phase end; with two
// exchange rows (by phase parity) neither can then overwrite a row the other still has to read.
//
// Per seam: the DP and the argmin of the owned last-row columns (atomic minimum), a team barrier,
// then every member hops through the phase ancestors itself, each wave of the team walks the
// phases its equal share of the rows touches from LDS windows of the 2-bit direction map and
// removes its rows (pixels right of the seam one column left), and a second team barrier.  Teams sit on
// one XCD (checked at start; a misplaced team flags the image).
#include "sc_device.h"

namespace sc {
namespace fwt {

constexpr int NT = kFwtThreads;  // 256
constexpr int NW = NT / 64;
constexpr int CPL = 4;
constexpr int XG = 8;                       // ghost columns on each side of a wave's core
constexpr int CORE = 64 * CPL - 2 * XG;     // 240 exact columns per wave
constexpr int WIN = NW * CORE + 2 * XG;     // 976 columns a member computes
constexpr int K = kFwtPhaseRows;            // 56 rows per phase
constexpr int XP = 2;                       // phases between two exchanges of the members' keys
constexpr int X = XP * K;                   // 112 ghost columns on each side of a member's owned range
constexpr int S = WIN - 2 * X;              // 752 columns a member of a multi-member team owns
constexpr int PF = 8;                       // rows of pixels loaded ahead; also the LDS refresh period
constexpr int GK = K / 4;                   // 4-row direction groups per phase
constexpr int WD = 32;                      // window dwords per group: columns je-59 .. je+68
constexpr int PMAX = (kFwdMaxH + K - 1) / K;
constexpr uint32_t INF = 0xFFFFFFFFu;
static_assert(S == kFwtOwned && WIN == kFwtWindow && K % PF == 0 && K <= 63 && PF == XG, "tile shape");

struct Smem {
    uint32_t xs[2][NW][2][2 * CPL];  // core edges of each wave: [refresh parity][wave][left, right][8 keys]
    uint32_t win[NW][GK * WD];
    int jend[PMAX];
    unsigned long long red[NW];
    uint32_t cw[(252 / K + 1) * 128];  // the backtrack's windows of ancestor offsets, 512 bytes per phase
    int flag;
    int chain;  // jend[p] is final for every p >= chain
};

// tag of the keys published at global phase number n (seam k, phase p: n = k * P + p): 1..511,
// never the 0 of a cleared exchange row; two phases apart the tags differ
__device__ __forceinline__ uint32_t phase_tag(int n) { return 1u + (uint32_t)n % 511u; }

constexpr int kSc1 = 16;  // cache-policy bits of a buffer load: sc1 (skip the CU's L1, read the L2)

// lane l receives lane l-1's value (lane 0: 0) / lane l+1's value (lane 63: 0)
__device__ __forceinline__ uint32_t from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);
}

// Member geometry: the first column of its window and the columns it owns.
struct Cols {
    int base, own0, own1;
};
__device__ __forceinline__ Cols member_cols(int rank, int gd) {
    Cols c;
    if (gd == 1) {
        c.base = 0;
        c.own0 = 0;
        c.own1 = WIN - XG;  // columns from 0 are exact up to the last wave's right ghost
    } else {
        c.base = rank * S - X;
        c.own0 = rank * S;
        c.own1 = rank * S + S;
    }
    return c;
}

// DP members of an image of width W (the same for every seam: owned ranges are fixed columns)
__device__ __forceinline__ int dp_members(int W) { return W <= WIN - XG ? 1 : (W + S - 1) / S; }

struct Carver {
    // The DP of one seam on the current width w for member `rank`: directions of the owned
    // columns, their phase ancestors, and the atomic minimum of their last-row keys into *amin.
    // A neighbour that gives up waiting flags the image; the team barrier after the DP then
    // abandons it.
    static __device__ __forceinline__ void dp(const Img& d, Smem& sm, int rank, int gd, int w, int k, int P,
                                              unsigned long long* amin) {
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        const int H = d.H;
        const Cols cl = member_cols(rank, gd);
        const int j0 = cl.base + CORE * wv + CPL * lane;  // the lane's first column
        bool act[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) act[c] = j0 + c >= 0 && j0 + c < w;
        const bool any = act[0];  // j0 is a multiple of 4: a group is in the image iff its first column is
        // exact lanes: a wave's core, and the left ghost of the first wave when the window starts at
        // column 0 (nothing lies left of it)
        const bool exact = (lane >= XG / CPL && lane < 64 - XG / CPL) || (wv == 0 && cl.base == 0 && lane < XG / CPL);
        const bool owned = exact && j0 >= cl.own0 && j0 < cl.own1 && j0 < w;  // groups of 4 are owned whole
        const bool mghost = any && (j0 < cl.own0 || j0 >= cl.own1);         // refreshed from other members
        // the lane whose first column is w loads too: column w keeps a copy of the row's last pixel
        const uint32_t v0 = j0 >= 0 && j0 <= w ? (uint32_t)j0 * 4u : kBufDrop;
        const __amdgpu_buffer_rsrc_t rwk = make_rsrc(d.wk, (uint32_t)H * (uint32_t)d.wp + (uint32_t)kFwdSlack);
        const uint32_t gbytes = (uint32_t)d.db * 4u;
        const __amdgpu_buffer_rsrc_t rdir = make_rsrc(d.dirs, (uint32_t)((H + 3) >> 2) * gbytes);
        const uint32_t dvo = owned ? (uint32_t)j0 : kBufDrop;  // byte j0/4 of a row's direction bytes, x4
        uint8_t* const ancg = reinterpret_cast<uint8_t*>(d.anc);
        uint32_t* const xq = d.xq;
        const bool noL = j0 == 0;  // column 0 has no upper-left parent
        bool okR[CPL];             // the column has an upper-right parent
        uint32_t tagR[CPL];        // the upper-right candidate's tag, or all ones (INF) without that parent
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            okR[c] = j0 + c + 1 < w;
            tagR[c] = okR[c] ? 0x100u : INF;
        }
        const uint32_t infL = noL ? INF : 0u;  // column 0 has no upper-left parent

        v4u ring[PF];
        static_for<PF>([&](auto U) {
            constexpr int u = decltype(U)::value;
            ring[u] = __builtin_amdgcn_raw_buffer_load_b128(rwk, (int)v0, (int)((uint32_t)min(u, H - 1) * (uint32_t)d.wp),
                                                            kSc1);
        });
        uint32_t Sk[CPL], Pup[CPL], dacc = 0, dkeep = 0;
        int phase = 0;

        // end of a phase: the owned columns' ancestor offsets, then (every XP phases, not after the
        // last) the exchange of the keys at the member's outer ghost columns, then the offsets
        // restart
        auto phase_end = [&]() {
            if (owned) {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (act[c]) *gp(ancg + (size_t)phase * d.W + j0 + c) = (uint8_t)(Sk[c] & 0x7Fu);
            }
            if (gd > 1 && phase + 1 < P && phase % XP == XP - 1) {
                const uint32_t tag = phase_tag(k * P + phase);
                uint32_t* xr = xq + (size_t)((phase / XP) & 1) * d.xw + (j0 > 0 ? j0 : 0);
                // every lane's publish comes before any lane's wait in program order
                if (owned) {
                    const v4u o = {(Sk[0] & ~0x1FFu) | tag, (Sk[1] & ~0x1FFu) | tag, (Sk[2] & ~0x1FFu) | tag,
                                   (Sk[3] & ~0x1FFu) | tag};
                    *gp(reinterpret_cast<v4u*>(xr)) = o;
                }
                asm volatile("" ::: "memory");
                if (mghost) {
                    unsigned long long t0 = 0;
                    // plain buffer loads with the sc1 bit (an atomic load would make the compiler
                    // wait for every access in flight at later loads)
                    const __amdgpu_buffer_rsrc_t rxq = make_rsrc(xq, (uint32_t)(2 * d.xw) * 4u);
                    const uint32_t xo = (uint32_t)(xr - xq) * 4u;
                    for (int it = 0;; ++it) {
                        const v4u xv = __builtin_amdgcn_raw_buffer_load_b128(rxq, (int)xo, 0, kSc1);
                        const uint32_t x[CPL] = {xv[0], xv[1], xv[2], xv[3]};
                        bool ok = true;
#pragma unroll
                        for (int c = 0; c < CPL; ++c) ok = ok && (!act[c] || (x[c] & 0x1FFu) == tag);
                        if (ok) {
#pragma unroll
                            for (int c = 0; c < CPL; ++c) Sk[c] = x[c] & ~0x1FFu;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        if ((it & 63) == 63) {  // bounded: 10 s, or at once when the image failed
                            const unsigned long long now = wall_clock64();
                            if (t0 == 0) t0 = now;
                            if (now - t0 > 1000000000ull ||
                                (__hip_atomic_load(gp(d.status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                                 (kStatusTimeout | kStatusPlacement))) {
                                __hip_atomic_fetch_or(gp(d.status), kStatusTimeout, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                                break;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) Sk[c] = (Sk[c] & ~0x7Fu) | 64u;
            ++phase;
        };

        // every XG rows: the waves' ghost columns next to other waves take those waves' core keys
        auto refresh = [&](int i) {
            const int b = (i / PF) & 1;
            if (lane == XG / CPL || lane == XG / CPL + 1) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) sm.xs[b][wv][0][CPL * (lane - XG / CPL) + c] = Sk[c];
            }
            if (lane == 64 - 2 * (XG / CPL) || lane == 64 - 2 * (XG / CPL) + 1) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) sm.xs[b][wv][1][CPL * (lane - (64 - 2 * (XG / CPL))) + c] = Sk[c];
            }
            lds_barrier();
            if (wv > 0 && lane < XG / CPL) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) Sk[c] = sm.xs[b][wv - 1][1][CPL * lane + c];
            }
            if (wv < NW - 1 && lane >= 64 - XG / CPL) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) Sk[c] = sm.xs[b][wv + 1][0][CPL * (lane - (64 - XG / CPL)) + c];
            }
        };

        auto row = [&](auto U, int i, auto LAST) {
            constexpr int u = decltype(U)::value;
            constexpr bool last = decltype(LAST)::value;  // the block holds row H-1: no refill
            const v4u px = ring[u];
            if (!last) {
                ring[u] = __builtin_amdgcn_raw_buffer_load_b128(rwk, (int)v0,
                                                                (int)((uint32_t)min(i + PF, H - 1) * (uint32_t)d.wp), kSc1);
                __builtin_amdgcn_sched_barrier(0);  // keep the refill PF rows ahead of its use
            }
            // pixels j0-1 .. j0+4: the neighbours come from the lanes beside (the left one clamped
            // to column 0 at the image's left edge, the right one to the pixel itself past the row)
            uint32_t pc[CPL + 2];
            pc[1] = px[0];
            pc[2] = px[1];
            pc[3] = px[2];
            pc[4] = px[3];
            // the cross-lane shifts run in every lane (a lane left out of a DPP read would hand its
            // neighbour a zero), and only then is the clamped value selected
            const uint32_t lpx = from_left(pc[4]);
            pc[5] = from_right(pc[1]);
            pc[0] = noL ? pc[1] : lpx;
            // right neighbours: column w holds a copy of the last pixel, so the clamp at the row's
            // end needs no select
            uint32_t pr[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) pr[c] = pc[c + 2];
            uint32_t bits = 0;
            if (u == 0 && i == 0) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    Sk[c] = (__builtin_amdgcn_sad_u8(pc[c], pr[c], 0u) << 9) | 64u;
                    bits |= 1u << (2 * c);
                }
            } else {
                const uint32_t Sl = from_left(Sk[CPL - 1]), Sr = from_right(Sk[0]);
                uint32_t Sn[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const uint32_t pl = pc[c];
                    const uint32_t cu = __builtin_amdgcn_sad_u8(pl, pr[c], 0u);
                    const uint32_t sL = c == 0 ? Sl : Sk[c - 1];
                    const uint32_t sR = c == CPL - 1 ? Sr : Sk[c + 1];
                    uint32_t kL = (__builtin_amdgcn_sad_u8(Pup[c], pl, 0u) << 9) + sL;
                    if (c == 0) kL |= infL;
                    const uint32_t kU = Sk[c] | 0x80u;
                    const uint32_t kR = ((__builtin_amdgcn_sad_u8(Pup[c], pr[c], 0u) << 9) + sR) | tagR[c];
                    const uint32_t kk = min3u(kL, kU, kR);
                    Sn[c] = next_state(kk, cu);
                    bits |= ((kk >> 7) & 3u) << (2 * c);
                }
#pragma unroll
                for (int c = 0; c < CPL; ++c) Sk[c] = Sn[c];
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) Pup[c] = pc[c + 1];
            dacc |= (bits & 0xFFu) << (8 * (u & 3));
            if constexpr (!last) {
                // a full block stores its two groups together at its end (a store between the
                // pixel prefetches would make the next row's wait cover the loads issued after it)
                if constexpr (u == 3) {
                    dkeep = dacc;
                    dacc = 0;
                } else if constexpr (u == PF - 1) {
                    __builtin_amdgcn_raw_buffer_store_b32(dkeep, rdir, (int)dvo, (int)((uint32_t)((i - 4) >> 2) * gbytes), 0);
                    __builtin_amdgcn_raw_buffer_store_b32(dacc, rdir, (int)dvo, (int)((uint32_t)(i >> 2) * gbytes), 0);
                    dacc = 0;
                }
            } else if ((u & 3) == 3 || i == H - 1) {
                __builtin_amdgcn_raw_buffer_store_b32(dacc, rdir, (int)dvo, (int)((uint32_t)(i >> 2) * gbytes), 0);
                dacc = 0;
            }
            // phases are K rows and start at multiples of PF (K % PF == 0), so a phase ends on the
            // last row of a block, or at the image's last row; the LDS refresh closes every block
            if constexpr (u == PF - 1) {
                if (((i + 1) % K) == 0 || (last && i == H - 1)) phase_end();
                if (!(last && i == H - 1)) refresh(i);
            } else if constexpr (last) {
                if (i == H - 1) phase_end();
            }
        };
        int i0 = 0;
#pragma unroll 1
        for (; i0 + PF < H; i0 += PF)
            static_for<PF>([&](auto U) { row(U, i0 + decltype(U)::value, std::false_type{}); });
        static_for<PF>([&](auto U) {
            if (i0 + decltype(U)::value < H) row(U, i0 + decltype(U)::value, std::true_type{});
        });
        // argmin of the owned last-row columns: packed (M << 32 | column), leftmost minimum
        unsigned long long best = ~0ull;
        if (owned) {
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                if (act[c]) best = min(best, ((unsigned long long)(Sk[c] >> 9) << 32) | (unsigned)(j0 + c));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) best = min(best, (unsigned long long)__shfl_xor((long long)best, o));
        if (lane == 0) sm.red[wv] = best;
        __syncthreads();
        if (t == 0) {
            unsigned long long b = sm.red[0];
            for (int x = 1; x < NW; ++x) b = min(b, sm.red[x]);
            if (b != ~0ull) __hip_atomic_fetch_min(gp(amin), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // The seams of one image by team member `rank` of G.
    static __device__ __forceinline__ void carve(const Img& d, Smem& sm, int rank, int G) {
        const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
        const int H = d.H, nseams = d.W - d.target_w, P = (H + K - 1) / K;
        const int gd = dp_members(d.W);
        GAS Ctl* ctl = gp(reinterpret_cast<Ctl*>(d.amin));
        const bool timer = rank == 0 && t == 0;
        unsigned epoch = 0;
        if (G > 1) {
            // every member records its XCD: a team must share one L2
            if (t == 0)
                __hip_atomic_fetch_or(&ctl->xmask, 1u << (xcc_id() & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!team_sync<true>(d, epoch, G, &sm.flag)) return;
            const unsigned m = __hip_atomic_load(&ctl->xmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__popc(m) != 1) {
                if (t == 0)
                    __hip_atomic_fetch_or(gp(d.status), kStatusPlacement, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        } else {
            __syncthreads();
        }
        if (timer) ctl->t_begin = wall_clock64();
        int k = 0;
#pragma unroll 1
        for (; k < nseams; ++k) {
            const int w = d.W - k;
            unsigned long long* amin = d.amk + (k & 1);
            const unsigned long long tm0 = timer ? wall_clock64() : 0ull;
            // no phase end of this seam is known yet; the barriers of the DP and after it order this
            // reset after every walker of the previous seam and before any of this one
            if (t == 0) sm.chain = 0x7fffffff;
            // A member whose owned columns all lie beyond the current width has nothing to compute
            // (its ghost columns belong to its left neighbour) and takes no part in the exchange.
            // That keeps every exchange mutual: the left neighbour of a participating member always
            // waits for that member's keys too, so neither can run two phases ahead and overwrite a
            // double-buffered row the other has not read yet.
            if (rank < gd && (gd == 1 || rank * S < w)) dp(d, sm, rank, gd, w, k, P, amin);
            if (G > 1) {
                if (!team_sync<true>(d, epoch, G, &sm.flag)) return;
            } else {
                __syncthreads();
            }
            const unsigned long long tm1 = timer ? wall_clock64() : 0ull;
            const unsigned long long key = __hip_atomic_load(gp(amin), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (rank == 0 && t == 0) {
                if (d.costs_out) *gp(d.costs_out + k) = (long long)(key >> 32);
                // the next seam's argmin word; the team barrier after the removal orders this
                // reset before any member's minimum of seam k + 1
                __hip_atomic_store(gp(d.amk + ((k + 1) & 1)), ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // ---- backtrack, first hop (every member on its own): wave 0 goes phase by phase
            // through the ancestor offsets and publishes each phase end in LDS as soon as it is
            // known; a wave starts on one of its phases once that phase's end is there, bottom
            // phases first.  (sm.chain was set above every phase before the DP's barriers.)
            // A phase end lies within K columns of the one below it, so wave 0 loads the ancestor
            // offsets of CH phases at once (the 512 bytes of each row around the current column,
            // two dwords per lane, into LDS) and lane 0 takes CH hops from there: one memory round
            // trip per CH hops instead of one per hop.
            if (wv == 0) {
                constexpr int CH = 252 / K + 1;  // h * K + 3 < 256 for every hop h of a round
                const __amdgpu_buffer_rsrc_t ranc = make_rsrc(d.anc, ((uint32_t)P * (uint32_t)d.W + 3u) & ~3u);
                int je = min(max((int)(key & 0xFFFFFFFFu), 0), w - 1);
                if (lane == 0) {
                    sm.jend[P - 1] = je;
                    __hip_atomic_store(&sm.chain, P - 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                for (int p = P - 1; p >= 1; p -= CH) {
                    const int m = min(CH, p);
                    uint32_t v[CH][2];
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        // byte window [o, o + 512) of phase p - h's row, o = row + je - 256 rounded
                        // down to a dword; dwords before the array are dropped
                        const int o = (p - h) * d.W + je - 256;
                        const int oa = o >= 0 ? o & ~3 : -((-o + 3) & ~3);
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int bo = oa + 4 * (lane + 64 * q);
                            v[h][q] = buf_ld32<true>(ranc, h < m && bo >= 0 ? (uint32_t)bo : kBufDrop);
                        }
                    }
#pragma unroll
                    for (int h = 0; h < CH; ++h) {
                        sm.cw[h * 128 + lane] = v[h][0];
                        sm.cw[h * 128 + 64 + lane] = v[h][1];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (lane == 0) {
                        const uint8_t* cb = reinterpret_cast<const uint8_t*>(sm.cw);
                        const int j0 = je;
                        for (int h = 0; h < m; ++h) {
                            const int o = (p - h) * d.W + j0 - 256;
                            const int oa = o >= 0 ? o & ~3 : -((-o + 3) & ~3);
                            je = min(max(je + (int)cb[h * 512 + (p - h) * d.W + je - oa] - 64, 0), w - 1);
                            sm.jend[p - 1 - h] = je;
                            __hip_atomic_store(&sm.chain, p - 1 - h, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                    je = __builtin_amdgcn_readfirstlane(je);  // lane 0's column, after its LDS reads
                    __builtin_amdgcn_wave_barrier();
                }
            }
            // ---- every wave of the team owns an equal range of rows [ra, rb) (waves numbered across
            // the team first); it walks each phase its range touches from an LDS window of the
            // direction map, bottom phase first as phase ends become known, and removes its rows
            const int TW = G * NW, tw = wv * G + rank;
            const int rpw = (H + TW - 1) / TW;
            const int ra = min(H, tw * rpw), rb = min(H, ra + rpw);
            const __amdgpu_buffer_rsrc_t rdw = make_rsrc(d.dirs, (uint32_t)((H + 3) >> 2) * (uint32_t)d.db * 4u);
#pragma unroll 1
            for (int p = (rb - 1) / K; ra < rb && p >= ra / K; --p) {
                while (__hip_atomic_load(&sm.chain, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) > p)
                    __builtin_amdgcn_s_sleep(1);
                const int r0 = p * K, n = min(K, H - r0), ng = (n + 3) >> 2;
                const int ia = max(ra, r0) - r0, ib = min(rb, r0 + n) - r0;  // this wave's rows of the phase
                const int je = sm.jend[p];
                const int cb0 = max(0, je - (K - 1)) >> 2;
                uint32_t* win = sm.win[wv];
                constexpr int NI = (GK * WD + 63) / 64;
                uint32_t v[NI];
                // buffer loads with the sc1 bit at 32-bit offsets, dropped outside the map and above
                // the wave's first group: no branches, so all of them go out before the first wait
#pragma unroll
                for (int mi = 0; mi < NI; ++mi) {
                    const int x = lane + 64 * mi, g = x / WD, qd = x % WD;
                    const uint32_t off = g >= (ia >> 2) && g < ng && cb0 + qd < d.db
                                             ? ((uint32_t)((r0 >> 2) + g) * (uint32_t)d.db + (uint32_t)(cb0 + qd)) * 4u
                                             : kBufDrop;
                    v[mi] = buf_ld32<true>(rdw, off);
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
                for (int i = n - 1; i >= ia; --i) {
                    if (lane == i) mys = s;
                    if (i > 0) {
                        const int qd = min(max((s >> 2) - cb0, 0), WD - 1);
                        const uint32_t wd = win[(i >> 2) * WD + qd];
                        s += (int)((wd >> ((i & 3) * 8 + (s & 3) * 2)) & 3u) - 1;
                        s = min(max(s, 0), w - 1);
                    }
                }
                if (lane >= ia && lane < ib && d.seams_out) *gp(d.seams_out + (size_t)k * H + r0 + lane) = mys;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // removal: in each row the pixels right of the seam move one column left, four
                // rows per memory round trip
#pragma unroll 1
                for (int i = ia; i < ib; i += 4) {
                    auto seg = [&](int q) {
                        SSeg g;
                        if (i + q >= ib) {
                            g.base = d.wk;
                            g.q0 = g.q1 = g.sh = g.n = 0;
                            return g;
                        }
                        const int si = min(max(__builtin_amdgcn_readlane(mys, i + q), 0), w - 1);
                        uint8_t* r = d.wk + (long long)(r0 + i + q) * d.wp;
                        // columns si+1 .. w move left, the copy of the last pixel at w included,
                        // so column w-1 then holds a copy of the new last pixel
                        return sseg<false>(r + (long long)si * 4, r + (long long)w * 4, 4);
                    };
                    shift_rows2_wave<2, false, false>(seg(0), seg(1), seg(2), seg(3), lane);
                    // a seam at the last column removed the pixel the copy repeated: the new last
                    // pixel (w-2) is copied to w-1 (after the shift's store to it, same wave)
                    const int sq = __shfl(mys, min(i + lane, 63), 64);  // row i + lane's seam, in lanes 0..3
                    if (lane < 4 && i + lane < ib && w >= 2) {
                        const int si = min(max(sq, 0), w - 1);
                        if (si == w - 1) {
                            uint32_t* r = reinterpret_cast<uint32_t*>(d.wk + (long long)(r0 + i + lane) * d.wp);
                            *gp(r + w - 1) = *gp(r + w - 2);
                        }
                    }
                }
            }
            if (G > 1) {
                if (!team_sync<true>(d, epoch, G, &sm.flag)) return;
            } else {
                __syncthreads();
            }
            if (timer) {
                const unsigned long long tm2 = wall_clock64();
                ctl->t_stage[0] += tm1 - tm0;
                ctl->t_stage[1] += tm2 - tm1;
            }
        }
        // ---- the carved rows go from the dword pixels of wk to img (C bytes each): the rows of
        // this member's phases, one wave per row
        if (nseams > 0) {
            const int tw = d.target_w, C = d.C;
#pragma unroll 1
            for (int p = rank; p < P; p += G) {
                const int r0 = p * K, r1 = min(H, r0 + K);
#pragma unroll 1
                for (int r = r0 + wv; r < r1; r += NW) {
                    const uint32_t* src = reinterpret_cast<const uint32_t*>(d.wk + (long long)r * d.wp);
                    uint8_t* dst = d.img + (long long)r * d.pitch;
                    for (int x = lane; x < tw; x += 64) {
                        const uint32_t px = ld<true>(src + x);
                        for (int c = 0; c < C; ++c) *gp(dst + (long long)x * C + c) = (uint8_t)(px >> (8 * c));
                    }
                }
            }
        }
        if (G > 1) {
            team_sync<true>(d, epoch, G, &sm.flag);
        } else {
            __syncthreads();
        }
        if (rank == 0 && t == 0) {
            ctl->done = (unsigned)k;
            ctl->t_end = wall_clock64();
        }
    }
};

}  // namespace fwt

// Batched forward carve: block b is member blk[b].y of the team of image blk[b].x (-1: no work).
// Single image: the team's members are blocks xcd, xcd + 8, ... (the others exit at once).
__global__ __launch_bounds__(fwt::NT, 3) void fwt_carve_kernel(const Img* __restrict__ imgs,
                                                               const int2* __restrict__ blk, int xcd) {
    __shared__ fwt::Smem sm;
    int2 me;
    if (blk) {
        me = blk[blockIdx.x];
    } else {
        if ((int)(blockIdx.x & 7) != xcd) return;
        me = make_int2(0, (int)(blockIdx.x >> 3));
    }
    if (me.x < 0) return;
    const Img d = imgs[me.x];
    if (me.y >= d.G) return;
    fwt::Carver::carve(d, sm, me.y, d.G);
}

// Copy-in for the forward carve: every pixel of src (or img) as one dword of wk (channels in the
// low bytes), control words reset, exchange rows cleared, and src copied to img when nothing is
// carved.  Grid: (workgroups per image, images).
template <int C>
__device__ void fwt_prepare_rows(const Img& d, const uint8_t* srcimg, int row0, int rstep) {
    const int W = d.W;
    const bool identity = d.src && d.target_w == d.W;
    for (int y = row0; y < d.H; y += rstep) {
        uint32_t* wr = reinterpret_cast<uint32_t*>(d.wk + (long long)y * d.wp);
        for (int x0 = 4 * (int)threadIdx.x; x0 < W; x0 += 4 * (int)blockDim.x) {
            SrcRow<C> r;
            r.load(srcimg, d.pitch, W, y, x0);
            if (x0 + 3 < W) {
                *gp(reinterpret_cast<v4u*>(wr + x0)) = v4u{r.px(0), r.px(1), r.px(2), r.px(3)};
            } else {
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (x0 + p < W) *gp(wr + x0 + p) = r.px(p);
            }
            // column W keeps a copy of the last pixel (the DP's right neighbour at the row's end)
            if (x0 + 4 >= W) {
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (x0 + p == W - 1) *gp(wr + W) = r.px(p);
            }
            if (identity) {
                uint8_t* o = d.img + (long long)y * d.pitch + (long long)x0 * C;
#pragma unroll
                for (int b = 0; b < 4 * C; ++b)
                    if (x0 * C + b < W * C) *gp(o + b) = (uint8_t)(r.r[1 + (b >> 2)] >> (8 * (b & 3)));
            }
        }
    }
}

__global__ __launch_bounds__(256) void fwt_prepare_kernel(const Img* __restrict__ imgs, int n) {
    const int i = blockIdx.y;
    if (i >= n) return;
    const Img d = imgs[i];
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            reset_ctl(d);
            *gp(d.amk) = *gp(d.amk + 1) = ~0ull;
        }
        for (int x = threadIdx.x; x < 2 * d.xw; x += blockDim.x) *gp(d.xq + x) = 0u;
    }
    const uint8_t* srcimg = d.src ? d.src : d.img;
    switch (d.C) {
        case 1: fwt_prepare_rows<1>(d, srcimg, blockIdx.x, gridDim.x); break;
        case 2: fwt_prepare_rows<2>(d, srcimg, blockIdx.x, gridDim.x); break;
        case 3: fwt_prepare_rows<3>(d, srcimg, blockIdx.x, gridDim.x); break;
        default: fwt_prepare_rows<4>(d, srcimg, blockIdx.x, gridDim.x); break;
    }
}

hipError_t launch_fwt_prepare(const Img* imgs, int n, int max_rows, hipStream_t st) {
    const int per = max_rows < 256 ? max_rows : 256;
    hipLaunchKernelGGL(fwt_prepare_kernel, dim3(per, n), dim3(256), 0, st, imgs, n);
    return hipGetLastError();
}

hipError_t launch_fwt_carve(const Img* imgs, const int2* blk, int nblocks, int xcd, hipStream_t st) {
    hipLaunchKernelGGL(fwt_carve_kernel, dim3(nblocks), dim3(fwt::NT), 0, st, imgs, blk, xcd & 7);
    return hipGetLastError();
}

int fwt_blocks_per_cu() {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwt_carve_kernel, fwt::NT, 0) == hipSuccess ? nb : 0;
}

}  // namespace sc
