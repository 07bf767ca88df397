// Device helpers shared by the kernels of libseamcarve (gfx950): global-address-space casts,
// raw buffer descriptors, the in-place row shifters, packed-pixel row loads and small VALU
// idioms.  Included by the .hip sources only.
#pragma once
#include <type_traits>
#include <utility>

#include "sc_internal.h"

namespace sc {

#define GAS __attribute__((address_space(1)))
// Every pointer reaches the kernels inside a descriptor, i.e. as a generic pointer; casting it to
// the global address space lets the compiler emit global_* instead of flat_* memory instructions.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ GAS T* gp(T* p) {
    return (GAS T*)p;
}

// Load of data that another workgroup of the same team may have written since this CU last read
// it.  A relaxed device-scope atomic load is a plain load with the sc1 cache bit: it skips the
// CU's L1 and reads the XCD's L2, where the other workgroup's stores have landed (a team always
// runs on one XCD).  Single-workgroup carves use ordinary loads.
template <bool COH, class T>
__device__ __forceinline__ T ld(const T* p) {
    if constexpr (COH)
        return __hip_atomic_load(gp(const_cast<T*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *gp(p);
}

// Raw buffer descriptors (gfx9 word 3).  A raw buffer access adds a wave-uniform byte offset
// (scalar register) to a per-lane byte offset (vector register); only the per-lane part is
// range checked, and an access whose per-lane offset is >= the descriptor's size is dropped
// (loads return 0, stores write nothing).
constexpr int kBufWord3 = 0x00020000;
constexpr uint32_t kBufDrop = 0x80000000u;  // a per-lane offset beyond any descriptor used here
typedef unsigned int v2u __attribute__((__vector_size__(8)));
typedef unsigned int v4u __attribute__((__vector_size__(16)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kBufWord3);
}

// A dword at a lane's byte offset into a buffer; COH sets the sc1 bit (the load reads the XCD's L2,
// like ld<true>).  Being a plain load, it leaves the compiler's memory-counter waits for later
// loads exact, where an atomic load in flight makes it wait for every outstanding access.
template <bool COH>
__device__ __forceinline__ uint32_t buf_ld32(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, COH ? 16 : 0);
}

template <bool COH>
__device__ __forceinline__ uint8_t buf_ld8(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, 0, COH ? 16 : 0);
}

__device__ __forceinline__ uint32_t xcc_id() {
    uint32_t v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v;
}

// Calls f(std::integral_constant<int, 0>{}) ... f(std::integral_constant<int, N-1>{}) in order.
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// One segment of a one-pixel shift inside a row, as 16-byte destination slots aligned to absolute
// addresses.  Left (R = false): destination [lo, hi) takes the bytes sh above it.  Right (R =
// true): destination [lo + sh, hi + sh) takes the bytes of [lo, hi).  A slot's output needs its
// own 16 bytes and one dword beyond it (above for left, below for right) that belongs to the
// neighbouring slot; slots are numbered so that pass order visits that neighbour in the same
// pass or a later one (left: ascending addresses, right: descending), and a pass loads before it
// stores, so the update is hazard free.
//
// The row must start on a 16-byte boundary and belong to the calling wave alone while it runs:
// a slot at either end of the destination is then written whole, with the bytes outside the
// destination put back as loaded.
struct SSeg {
    uint8_t* base;  // 16-byte aligned
    int q0, q1;     // destination bytes [base + q0, base + q1)
    int sh;         // shift in bytes, 1..4
    int n;          // slots
};

template <bool R>
__device__ __forceinline__ SSeg sseg(uint8_t* lo, uint8_t* hi, int sh) {
    SSeg g;
    uint8_t* dlo = R ? lo + sh : lo;
    const int off = (int)((uintptr_t)dlo & 15);
    g.base = dlo - off;
    g.q0 = off;
    g.q1 = hi > lo ? off + (int)(hi - lo) : off;
    g.sh = sh;
    g.n = g.q1 > g.q0 ? ((g.q1 - 1) >> 4) + 1 : 0;
    return g;
}

// W[u] holds 20 loaded bytes: left = the slot then the dword above, right = the dword below then
// the slot.  The accesses are buffer loads and stores through a descriptor starting 16 bytes below
// the segment's first slot, so every offset is non-negative; a lane without a slot, or without a
// neighbour dword to read, gets a dropped offset (its load returns 0, its store writes nothing).
// With no branches around them, all loads of a pass go out before the first wait.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sseg_rsrc(const SSeg& g) {
    return make_rsrc(g.base - 16, (uint32_t)(g.n + 2) * 16u);
}

template <int U, bool R>
__device__ __forceinline__ void sseg_load(const SSeg& g, int fb, int lane, uint32_t (&W)[U][5]) {
    const __amdgpu_buffer_rsrc_t r = sseg_rsrc(g);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = fb + u * 64 + lane;
        const bool in = f < g.n;
        const int so = (R ? g.n - 1 - f : f) << 4;
        const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(in ? (uint32_t)so + 16u : kBufDrop), 0, 0);
        constexpr int k = R ? 1 : 0;
        W[u][k + 0] = v[0]; W[u][k + 1] = v[1];
        W[u][k + 2] = v[2]; W[u][k + 3] = v[3];
        if (R) {
            const bool nb = in && so > g.q0 - g.sh;
            W[u][0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(nb ? (uint32_t)so + 12u : kBufDrop), 0, 0);
        } else {
            const bool nb = in && so + 16 - g.sh < g.q1;
            W[u][4] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(nb ? (uint32_t)so + 32u : kBufDrop), 0, 0);
        }
    }
}

template <int U, bool R>
__device__ __forceinline__ void sseg_store(const SSeg& g, int fb, int lane, const uint32_t (&W)[U][5]) {
    const __amdgpu_buffer_rsrc_t r = sseg_rsrc(g);
    const int a = R ? 4 - g.sh : g.sh;  // byte offset of the output inside the 20 bytes
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = fb + u * 64 + lane;
        const int so = (R ? g.n - 1 - f : f) << 4;
        uint32_t o[4];
        if (a == 4) {
            o[0] = W[u][1]; o[1] = W[u][2]; o[2] = W[u][3]; o[3] = W[u][4];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbyte(W[u][i + 1], W[u][i], (uint32_t)a);
        }
        if (so < g.q0 || so + 16 > g.q1) {
            // an end slot: bytes outside the destination keep the values the pass loaded
            const int c0 = min(max(g.q0 - so, 0), 16), c1 = min(max(g.q1 - so, 0), 16);
            const uint32_t m16 = ((1u << c1) - 1u) & ~((1u << c0) - 1u);  // bit k = byte k of the slot
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t bm = ((((m16 >> (4 * i)) & 15u) * 0x00204081u) & 0x01010101u) * 0xffu;
                const uint32_t cur = R ? W[u][i + 1] : W[u][i];
                o[i] = (o[i] & bm) | (cur & ~bm);
            }
        }
        const v4u ov = {o[0], o[1], o[2], o[3]};
        __builtin_amdgcn_raw_buffer_store_b128(ov, r, (int)(f < g.n ? (uint32_t)so + 16u : kBufDrop), 0, 0);
    }
}

// Two rows' shifts (image and energy segments of row a, then of row b, directions RA and RB)
// moved together: every pass issues the loads of all four segments before any store, so the
// rows share each memory round trip.  The segments must not overlap each other's bytes.
template <int U, bool RA, bool RB>
__device__ __forceinline__ void shift_rows2_wave(const SSeg& a0, const SSeg& a1, const SSeg& b0, const SSeg& b1,
                                                 int lane) {
    const int n = max(max(a0.n, a1.n), max(b0.n, b1.n));
#pragma unroll 1
    for (int fb = 0; fb < n; fb += 64 * U) {
        uint32_t W0[U][5], W1[U][5], W2[U][5], W3[U][5];
        sseg_load<U, RA>(a0, fb, lane, W0);
        sseg_load<U, RA>(a1, fb, lane, W1);
        sseg_load<U, RB>(b0, fb, lane, W2);
        sseg_load<U, RB>(b1, fb, lane, W3);
        sseg_store<U, RA>(a0, fb, lane, W0);
        sseg_store<U, RA>(a1, fb, lane, W1);
        sseg_store<U, RB>(b0, fb, lane, W2);
        sseg_store<U, RB>(b1, fb, lane, W3);
    }
}

// dst bytes [dst, dst + n) take the bytes of [src, src + n), one wave; the buffers do not overlap.
// Dword-granular on the destination; bytes of a destination dword outside [dst, dst + n) are not
// written (they may belong to a neighbouring row).  Source dwords may be read a few bytes beyond
// either end of the source range.
__device__ __forceinline__ void copy_bytes_wave(uint8_t* dst, const uint8_t* src, int n, int lane) {
    if (n <= 0) return;
    const int off = (int)((uintptr_t)dst & 3);
    uint8_t* const base = dst - off;  // dword-aligned; destination dword j covers base + 4j
    const int nd = ((off + n - 1) >> 2) + 1;
    const uintptr_t s0 = (uintptr_t)src - (uintptr_t)off;  // source byte of base + x is s0 + x
#pragma unroll 1
    for (int jb = 0; jb < nd; jb += 64 * 4) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = jb + u * 64 + lane;
            v[u] = 0;
            if (j < nd) {
                const uintptr_t sa = s0 + 4 * (uintptr_t)j;
                const uint32_t* sp = reinterpret_cast<const uint32_t*>(sa & ~(uintptr_t)3);
                const uint32_t lo = *gp(sp);
                const uint32_t hi = (sa & 3) ? *gp(sp + 1) : 0u;
                v[u] = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(sa & 3));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = jb + u * 64 + lane;
            if (j >= nd) continue;
            uint8_t* dp = base + 4 * j;
            if (dp >= dst && dp + 4 <= dst + n) {
                *gp(reinterpret_cast<uint32_t*>(dp)) = v[u];
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (dp + k >= dst && dp + k < dst + n) *gp(dp + k) = (uint8_t)(v[u] >> (8 * k));
            }
        }
    }
}

// ----------------------------------------------------------------------------------------------
// Single-workgroup DP helpers (forward energy, object removal).

// v_min3_u32: the smallest of three tagged keys (ties go to the smallest tag, i.e. the leftmost).
__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t o;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(o) : "v"(a), "v"(b), "v"(c));
    return o;
}

// kk + (cu << 9) - 127 * tag - 1 with tag = bits 7-8 of kk: drops the tag, adds CU to M and moves
// the ancestor offset by tag - 1.
__device__ __forceinline__ uint32_t next_state(uint32_t kk, uint32_t cu) {
    const uint32_t tag = (kk >> 7) & 3u;
    uint32_t o;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(o) : "v"(tag), "s"(-127), "v"(kk + (cu << 9) - 1u));
    return o;
}

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The pixels a thread needs from one row of a working image: CPL columns j0 .. j0+CPL-1 and one
// neighbour on each side, as packed channels.
template <int C, int CPL>
struct PixRow {
    // A thread reads the dwords covering columns j0-1 .. j0+CPL of a row: they start at byte
    // j0*C - 4 (j0*C is a multiple of 4 because CPL is), where column j0-1 sits at byte LEAD.
    static constexpr int LEAD = (4 - C % 4) % 4;
    static constexpr int NDW = (LEAD + (CPL + 2) * C + 3) / 4;
    static constexpr uint32_t PMASK = C == 4 ? 0xFFFFFFFFu : (1u << (8 * C)) - 1u;
    static_assert(CPL % 4 == 0, "a thread's directions fill whole bytes");

    // vl: byte offset of the dword left of column j0 (it holds only column j0-1); v0: of column j0.
    // Either is kBufDrop where nothing may be read (the load then returns 0).
    static __device__ __forceinline__ void load_row(uint32_t (&v)[NDW], __amdgpu_buffer_rsrc_t r, uint32_t vl,
                                                    uint32_t v0, uint32_t soff) {
        v[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)vl, (int)soff, 0);
#pragma unroll
        for (int q = 1; q < NDW; ++q) v[q] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(v0 + 4u * (q - 1)), (int)soff, 0);
    }

    // pixel k (column j0-1+k) of a loaded row, channels packed in the low bytes
    static __device__ __forceinline__ void pixels(const uint32_t (&v)[NDW], uint32_t (&p)[CPL + 2]) {
#pragma unroll
        for (int k = 0; k < CPL + 2; ++k) {
            const int o = LEAD + C * k, q = o >> 2, r = o & 3;
            uint32_t x;
            if (r == 0) x = v[q];
            else if (r + C <= 4) x = v[q] >> (8 * r);
            else x = __builtin_amdgcn_alignbyte(v[q + 1], v[q], (uint32_t)r);
            p[k] = x & PMASK;
        }
    }

};

// ----------------------------------------------------------------------------------------------
// Team barrier.  One workgroup: a workgroup barrier.  A team of G workgroups on one XCD: each
// thread waits for its own stores to reach the L2 (vmcnt), then one thread per workgroup bumps
// the image's counter with a device-scope atomic and polls it with device-scope loads until all
// G have arrived; readers then fetch shared data with sc1 loads (see ld<true>).  The wait is
// bounded: after ~10 s it flags the image and every member gives up on it.
template <bool TEAM>
__device__ __forceinline__ bool team_sync(const Img& d, unsigned& epoch, int G, int* flag) {
    if constexpr (!TEAM) {
        __syncthreads();
        return true;
    } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) {
            epoch += (unsigned)G;
            __hip_atomic_fetch_add(gp(d.bar), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long t0 = wall_clock64();
            int ab = 0;
            while (__hip_atomic_load(gp(d.bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (__hip_atomic_load(gp(d.status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                    (kStatusTimeout | kStatusPlacement)) {
                    ab = 1;
                    break;
                }
                if (wall_clock64() - t0 > 1000000000ull) {  // 10 s at the 100 MHz constant clock
                    __hip_atomic_fetch_or(gp(d.status), kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ab = 1;
                    break;
                }
            }
            *flag = ab;
        }
        __syncthreads();
        return *flag == 0;
    }
}

// Reset the control words of one image (every carve launch starts from them).
__device__ __forceinline__ void reset_ctl(const Img& d) {
    GAS Ctl* c = gp(reinterpret_cast<Ctl*>(d.amin));
    c->amin = ~0ull;
    c->bar = 0;
    c->status = 0;
    c->t_begin = c->t_end = 0;
    c->xmask = 0;
    c->done = 0;
    c->t_stage[0] = c->t_stage[1] = c->t_stage[2] = 0;
    c->ebase = 0;
    c->stop = 0;
}

// One source row as seen by a thread owning 4 pixels from column x0: the aligned dwords covering
// the pixels and one neighbour on each side, realigned to the row's start with v_alignbyte (a
// caller's rows may start at any byte).
template <int C>
struct SrcRow {
    static constexpr int ND = C + 3;   // dwords loaded per thread
    static constexpr uint32_t PMASK = C == 4 ? 0xFFFFFFFFu : (1u << (8 * C)) - 1u;
    uint32_t r[C + 2];                 // row bytes [x0*C - 4, x0*C + 4*C + 4), dword aligned to the row

    // Row y of the image (pitch bytes per row, W*C bytes used): the thread's pixels start at x0.
    __device__ __forceinline__ void load(const uint8_t* img, long long pitch, int W, int y, int x0) {
        const uint8_t* row = img + (long long)y * pitch;
        const uint32_t sh = (uint32_t)((uintptr_t)row & 3u);
        // the descriptor covers the whole dwords holding the row's bytes (a dword-aligned dword that
        // holds an image byte lies inside the image's allocation); dwords outside are dropped (read
        // as 0), and only clamped neighbours would use them
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(row - sh, (sh + (uint32_t)(W * C) + 3u) & ~3u);
        // per-lane offsets never wrap: the dword left of column x0 has an offset of its own (dropped
        // at x0 = 0), the others count up from column x0 (an immediate offset may be folded in)
        const uint32_t v0 = x0 < W ? (uint32_t)(x0 * C) : kBufDrop;
        const uint32_t vl = x0 < W && x0 > 0 ? (uint32_t)(x0 * C - 4) : kBufDrop;
        uint32_t d[ND];
        d[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vl, 0, 0);
#pragma unroll
        for (int m = 1; m < ND; ++m) d[m] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(v0 + 4u * (m - 1)), 0, 0);
#pragma unroll
        for (int m = 0; m < C + 2; ++m) r[m] = __builtin_amdgcn_alignbyte(d[m + 1], d[m], sh);
    }
    // pixel p of the thread (p = -1 .. 4), channels packed in the low bytes
    __device__ __forceinline__ uint32_t px(int p) const {
        const int o = 4 + p * C, q = o >> 2, b = o & 3;
        const uint32_t v = b == 0 ? r[q] : __builtin_amdgcn_alignbyte(r[q + 1], r[q], (uint32_t)b);
        return v & PMASK;
    }
};

}  // namespace sc
