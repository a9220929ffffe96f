// Step, read-out and set-up kernels of the lattice Boltzmann library.
//
// One thread updates one cell; cells are numbered i = (x*ny + y)*nz + z
// (Sec. 2.5), so a wavefront covers 64 consecutive z and every population
// stream is read and written as contiguous runs (SoA). Flags carry the cell
// type in bits 0-1 and two hints: FL_BORDER (fluid cell on a box face, whose
// neighbours may wrap) and FL_NEARWALL (fluid cell with a non-fluid
// neighbour). Cells without hints take the fast path: neighbour i + d_k, no
// flag look-ups, no bounce-back branch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "collide.hpp"
#include "internal.hpp"

namespace lbm {

template <class ST>
using real_t = typename ST::R;

// Cache policy of the population streams of the step kernels. Each value is
// read once and written once per step, yet nontemporal hints measured slower
// on gfx950 (the lines a misaligned neighbour access shares with the next
// wave get evicted early), so both are off by default.
#ifndef LBM_NT_LOADS
#define LBM_NT_LOADS 0
#endif
#ifndef LBM_NT_STORES
#define LBM_NT_STORES 0
#endif
// Map consecutive blocks of the step kernels to one XCD's contiguous share of
// the lattice (blocks are dealt round-robin over the 8 XCDs).
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 0
#endif

// Population accessor. SoA addresses are formed as a wave-uniform 64-bit
// base (array + k * stride + shift, kept in scalar registers) plus one 32-bit
// lane offset i * sizeof(T) shared by every stream, so the 19 or 27 streams
// of a cell cost a single address register. The SoA array carries a halo of
// padding around its streams (see the runtime), so a shifted access i + d for
// any cell of the box stays inside the allocation; lanes that will not store
// may therefore load speculatively without clamping. The blocked layout keeps
// the Q streams of each run of kBlockCells cells together: value (k, j) at
// ((j / B) Q + k) B + j mod B, counted from the allocation's start, where
// cell i sits at j = i + P and P, whole blocks of padding that cover the
// largest neighbour offset, is passed in `stride`; offsets are 32-bit (the
// runtime keeps such arrays below 4 GiB).
// A value rounded to the storage type. On its way into FP16 the float passes
// an empty asm, which makes it opaque to the compiler: the operation that
// produced it can then not be folded with the conversion into one
// mixed-precision instruction with an FP16 result (v_fma_mixlo_f16 rounds
// a * b + c to FP16 once, where the FP32 arithmetic followed by the
// conversion rounds twice). Without it, two kernels holding the same float
// could store different FP16 bits, depending on instruction selection.
template <class ST>
__device__ __forceinline__ typename ST::T to_storage(real_t<ST> v)
{
    if constexpr (sizeof(typename ST::T) == 2) asm volatile("" : "+v"(v));
    return typename ST::T(v);
}

template <class ST, int LAYOUT, int Q, bool STREAM = false>
struct Acc {
    using T = typename ST::T;
    T* base;
    int64_t stride;
    __device__ __forceinline__ T* ptr_shift(uint32_t i, int k, int64_t d) const
    {
        if constexpr (LAYOUT == LAYOUT_SOA) {
            char* b = reinterpret_cast<char*>(base + (int64_t)k * stride + d);
            return reinterpret_cast<T*>(b + (uint32_t)(i * (uint32_t)sizeof(T)));
        } else if constexpr (LAYOUT == LAYOUT_BLOCKED) {
            constexpr uint32_t B = kBlockCells;
            const uint32_t j = i + (uint32_t)(d + stride);
            const uint32_t idx = (j & ~(B - 1)) * (uint32_t)Q + (uint32_t)k * B + (j & (B - 1));
            return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T));
        } else {
            return base + ((int64_t)i + d) * Q + k;
        }
    }
    __device__ __forceinline__ T* ptr(uint32_t i, int k) const { return ptr_shift(i, k, 0); }
    __device__ __forceinline__ real_t<ST> ld(uint32_t i, int k) const { return real_t<ST>(raw_ld(i, k)); }
    __device__ __forceinline__ void st(uint32_t i, int k, real_t<ST> v) const { raw_st(i, k, to_storage<ST>(v)); }
    __device__ __forceinline__ T raw_ld(uint32_t i, int k) const { return raw_ld_shift(i, k, 0); }
    __device__ __forceinline__ void raw_st(uint32_t i, int k, T v) const { raw_st_shift(i, k, 0, v); }
    __device__ __forceinline__ T raw_ld_shift(uint32_t i, int k, int64_t d) const
    {
        if constexpr (STREAM && LBM_NT_LOADS) return __builtin_nontemporal_load(ptr_shift(i, k, d));
        else return *ptr_shift(i, k, d);
    }
    __device__ __forceinline__ void raw_st_shift(uint32_t i, int k, int64_t d, T v) const
    {
        if constexpr (STREAM && LBM_NT_STORES) __builtin_nontemporal_store(v, ptr_shift(i, k, d));
        else *ptr_shift(i, k, d) = v;
    }
    // Speculative load at i + d for the fast path: SoA and the blocked layout
    // rely on their padding; AoS (no halo) clamps the cell index into the box.
    __device__ __forceinline__ real_t<ST> ld_fast(uint32_t i, int k, int64_t d, uint32_t ntot) const
    {
        if constexpr (LAYOUT == LAYOUT_SOA || LAYOUT == LAYOUT_BLOCKED) {
            return real_t<ST>(raw_ld_shift(i, k, d));
        } else {
            const int64_t j = (int64_t)i + d;
            return real_t<ST>(raw_ld((uint32_t)(j < 0 ? 0 : (j >= (int64_t)ntot ? ntot - 1 : j)), k));
        }
    }
    __device__ __forceinline__ T raw_ld_fast(uint32_t i, int k, int64_t d, uint32_t ntot) const
    {
        if constexpr (LAYOUT == LAYOUT_SOA || LAYOUT == LAYOUT_BLOCKED) {
            return raw_ld_shift(i, k, d);
        } else {
            const int64_t j = (int64_t)i + d;
            return raw_ld((uint32_t)(j < 0 ? 0 : (j >= (int64_t)ntot ? ntot - 1 : j)), k);
        }
    }
};

struct Coord {
    int x, y, z;
};

__device__ __forceinline__ Coord cell_coord(uint32_t i, const Field& F)
{
    const uint32_t plane = (uint32_t)F.ny * (uint32_t)F.nz;
    Coord c;
    c.x = (int)(i / plane);
    const uint32_t r = i - (uint32_t)c.x * plane;
    c.y = (int)(r / (uint32_t)F.nz);
    c.z = (int)(r - (uint32_t)c.y * (uint32_t)F.nz);
    return c;
}

// Index corrections of the z-face lanes of the AA odd fast kernel in FP16. A
// lane on a z face (a wall cell, or a fluid cell that the edge part updates)
// never uses what it reads across that face, so it may read its own row
// instead: +1 at z = 0, -1 at z = nz - 1. The wave then touches no cache line
// of the neighbouring row. In FP16 a row of 256 cells spans four lines of a
// stream, and that line of the neighbouring row added a quarter to the reads
// of each z-shifted stream (AA odd: 361 -> 322 us per step on the 256^3
// cavity); in FP32 and FP64 the share is an eighth and a sixteenth, and the
// correction measured slower. z = i - nz floor(i / nz), the quotient being the
// high word of i * ceil(2^64 / nz); F.zrecip = 0 (nz < 2) turns it off.
__device__ __forceinline__ void face_rows(const Field& F, uint32_t i, int32_t& zp, int32_t& zm)
{
    if (!F.zrecip) return;
    const uint32_t row = (uint32_t)__umul64hi((unsigned long long)i, F.zrecip);
    const uint32_t z = i - row * (uint32_t)F.nz;
    zp = z == 0 ? 1 : 0;
    zm = z == (uint32_t)F.nz - 1 ? -1 : 0;
}

// Neighbour x + s*c_k. Interior cells: constant offset. Border cells: wrap
// each coordinate (only periodic axes ever wrap for a fluid cell).
template <int Q, int K, int SIGN>
__device__ __forceinline__ uint32_t neighbour(const Field& F, uint32_t i, bool border, const Coord& c)
{
    constexpr int cx = SIGN * L<Q>::cx(K), cy = SIGN * L<Q>::cy(K), cz = SIGN * L<Q>::cz(K);
    if (!border) return (uint32_t)((int64_t)i + (int64_t)cx * F.ny * F.nz + (int64_t)cy * F.nz + cz);
    int x = c.x + cx, y = c.y + cy, z = c.z + cz;
    x = x < 0 ? x + F.nx : (x >= F.nx ? x - F.nx : x);
    y = y < 0 ? y + F.ny : (y >= F.ny ? y - F.ny : y);
    z = z < 0 ? z + F.nz : (z >= F.nz ? z - F.nz : z);
    return ((uint32_t)x * (uint32_t)F.ny + (uint32_t)y) * (uint32_t)F.nz + (uint32_t)z;
}

template <int Q, int K, int SIGN>
__device__ __forceinline__ int32_t offset(const Field& F)
{
    constexpr int cx = SIGN * L<Q>::cx(K), cy = SIGN * L<Q>::cy(K), cz = SIGN * L<Q>::cz(K);
    return cx * F.ny * F.nz + cy * F.nz + cz;
}

__device__ __forceinline__ bool is_fluid(const Field& F, uint32_t j) { return (F.flags[j] & FL_TYPE) == FL_FLUID; }

// A population bounced back at the non-fluid cell j: pressure walls reflect
// it with the opposite sign (anti-bounce-back), the others as it is.
template <class R>
__device__ __forceinline__ R reflect(const Field& F, uint32_t j, R v)
{
    return (F.flags[j] & FL_TYPE) == FL_PRESSURE ? -v : v;
}

// Curved wall on the link from fluid cell x to the wall cell s = x - c_k at
// the fraction q of the link from x (linear interpolated bounce-back in pull
// form; q = 1/2 is the half-way wall): the population entering x in
// direction k from the post-collision values f_out_kbar(x), f_out_k(x),
// f_out_kbar(x + c_k) (the value streaming in along the same line from the
// other side; f_out_kbar(x) when x + c_k is not fluid) and the wall term w.
template <class R>
__device__ __forceinline__ R curved_link(double q, R fo_kbar_x, R fo_k_x, R fo_kbar_n, R w)
{
    if (q == 0.5) return fo_kbar_x + w;
    const R qq = R(q);
    if (q > 0.5) return (fo_kbar_x + (R(2) * qq - R(1)) * fo_k_x + w) / (R(2) * qq);
    return R(2) * qq * fo_kbar_x + (R(1) - R(2) * qq) * fo_kbar_n + w;
}

// Gathered population f_k(x) across the non-fluid cell s = x - c_k in pull
// form, from an array holding f_out_kbar in slot k (AA after an even step,
// 2Pop pull): slot k of x plus (or, at a pressure wall, minus) the wall's
// slot kbar; on a curved link the interpolated rule.
template <int Q, int K, class ST, class A>
__device__ __forceinline__ real_t<ST> gather_across(const Field& F, const A& a, uint32_t i, uint32_t s, bool border,
                                                    const Coord& c)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const R w = a.ld(s, S::opp(K));
    if (F.qlink && !((F.flags[s] & FL_TYPE) == FL_PRESSURE)) {
        const uint32_t n = neighbour<Q, K, 1>(F, i, border, c);
        const R own = a.ld(i, K);
        return curved_link<R>(F.qlink[(size_t)K * F.ntot + i], own, a.ld(i, S::opp(K)),
                              is_fluid(F, n) ? a.ld(n, K) : own, w);
    }
    return reflect(F, s, a.ld(i, K)) + w;
}

template <class R>
__device__ __forceinline__ Relax<R> relax_of(const RelaxD& p)
{
    return Relax<R>{R(p.omega), R(p.omega_m), R(p.omega_b), R(p.omega3), R(p.omega4)};
}

// Stored terms of a wall cell of the built-in geometries: the lid's terms on
// lid cells (from the host's table, in the storage type), zero on the walls
// at rest.
template <int Q, class ST, int K>
__device__ __forceinline__ real_t<ST> builtin_wall_term(const Field& F, uint8_t type)
{
    if (type != FL_LID) return real_t<ST>(0);
    if constexpr (sizeof(typename ST::T) == 8) return F.lid.d[K];
    else return F.lid.f[K];
}

// Loads never wait for the flag byte: every lane issues its population loads
// at once (lanes of wall cells read harmless values from inside the
// allocation), collides, and only the stores and the bounce-back gather of
// cells next to walls depend on the flag.
// An empty asm that takes the loaded values as operands: the loads must then
// be issued for every lane before the flag decides anything, instead of being
// sunk under the flag test (which serialises one memory latency per wave).
template <class R, int Q>
__device__ __forceinline__ void issue_all(R (&g)[Q])
{
#pragma unroll
    for (int k = 0; k < Q; ++k) asm volatile("" : "+v"(g[k]));
}


// Every step kernel exists in three parts. PART_FAST runs over all cells and
// updates the fluid cells whose neighbours are all fluid and inside the box
// (constant offsets, no bounce-back code, few registers). PART_SLOW runs over
// the list of the other fluid cells (next to a wall or on a periodic face)
// with the general neighbour and bounce-back logic. PART_ALL does both in one
// pass (used by the batched ensemble). Each cell touches its own set of
// memory locations, so the split does not change any result (Sec. 2.3).
enum Part { PART_ALL = 0, PART_FAST = 1, PART_SLOW = 2 };

// Wall-plane cells stay on the fast path: their non-fluid neighbours are
// exactly the nine on one side of the cell, the side with normal axis a and
// sign s given by the plane code 1 + 2a + (s > 0). For a direction k the
// neighbour x + c_k is then a wall iff c_k,a = s, and x - c_k iff c_k,a = -s.
// The fast kernels apply those bounce-backs under a per-lane predicate;
// waves without such lanes skip the branch.
template <int Q, int K>
__device__ __forceinline__ bool wall_to(uint8_t fl)  // x + c_k is a wall
{
    const int code = (fl & FL_PLANE) >> FL_PLANE_SHIFT;
    bool w = false;
    static_for<0, 3>([&](auto A) {
        constexpr int a = A;
        constexpr int c = L<Q>::c(K, a);
        if constexpr (c != 0) w = w || code == 1 + 2 * a + (c > 0 ? 1 : 0);
    });
    return w;
}

template <int Q, int K>
__device__ __forceinline__ bool wall_from(uint8_t fl)  // x - c_k is a wall
{
    return wall_to<Q, L<Q>::opp(K)>(fl);
}

// ---------------------------------------------------------------------------
// Double-population scheme (Table 1, row 2Pop): collide pop(x), push
// out_k(x + c_k) <- f_out_k, or out_kbar(x) <- f_out_k + pop_k(x + c_k) when
// the neighbour is a wall (whose pop_k holds the momentum-exchange term).
template <int Q, class ST, int LAYOUT>
__device__ __forceinline__ void push_2pop_slow(const Field& F, uint32_t i, uint8_t fl, const real_t<ST> (&g)[Q])
{
    using S = L<Q>;
    const Acc<ST, LAYOUT, Q, true> src{(typename ST::T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> dst{(typename ST::T*)F.out, F.stride};
    const bool border = fl & FL_BORDER;
    const Coord c = border ? cell_coord(i, F) : Coord{0, 0, 0};
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == S::rest) {
            dst.st(i, k, g[k]);
        } else {
            const uint32_t j = neighbour<Q, k, 1>(F, i, border, c);
            if (is_fluid(F, j)) dst.st(j, k, g[k]);
            else dst.st(i, S::opp(k), reflect(F, j, g[k]) + src.ld(j, k));
        }
    });
}

template <int Q, int MODEL, class ST, int LAYOUT, int PART>
__device__ __forceinline__ void cell_2pop(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> src{(typename ST::T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> dst{(typename ST::T*)F.out, F.stride};
    const uint8_t fl = F.flags[i];
    R g[Q];
    static_for<0, Q>([&](auto K) { g[K] = src.ld(i, K); });
    if constexpr (PART != PART_SLOW) issue_all(g);
    collide<Q, MODEL, ST::shifted>(g, p);
    if constexpr (PART == PART_SLOW) {
        push_2pop_slow<Q, ST, LAYOUT>(F, i, fl, g);
    } else {
        if ((fl & FL_TYPE) != FL_FLUID) return;
        if (!(fl & FL_SLOW)) {
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                if (!wall_to<Q, k>(fl)) {
                    dst.raw_st_shift(i, k, offset<Q, k, 1>(F), to_storage<ST>(g[k]));
                } else {  // out_kbar(x) <- f_out_k + pop_k(x + c_k)
                    const R w = R(src.raw_ld_shift(i, k, offset<Q, k, 1>(F)));
                    dst.st(i, L<Q>::opp(k), g[k] + w);
                }
            });
        } else if constexpr (PART == PART_ALL) {
            push_2pop_slow<Q, ST, LAYOUT>(F, i, fl, g);
        }
    }
}

// Swap algorithm, collision sweep (Table 1, row Swap): pop_kbar(x) <- f_out_k.
// Purely local, so every fluid cell is handled by the fast part. Lanes of
// wall cells store back the values they loaded (slot k̄ gets its own value),
// which changes nothing in memory but keeps every store instruction writing
// whole cache lines: a line left partly unwritten costs a read-modify-write
// in HBM.
template <int Q, int MODEL, class ST, int LAYOUT>
__device__ __forceinline__ void cell_swap_collide(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> a{(typename ST::T*)F.pop, F.stride};
    const uint8_t fl = F.flags[i];
    R g[Q], keep[Q];
    static_for<0, Q>([&](auto K) { g[K] = a.ld(i, K); });
    issue_all(g);
    static_for<0, Q>([&](auto K) { keep[K] = g[K]; });
    collide<Q, MODEL, ST::shifted>(g, p);
    const bool fluid = (fl & FL_TYPE) == FL_FLUID;
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        a.st(i, S::opp(k), fluid ? g[k] : keep[S::opp(k)]);
    });
}

// Swap algorithm, streaming sweep over k < rest: pop_kbar(x) <-> pop_k(x + c_k)
// with a fluid neighbour, pop_kbar(x) += pop_k(x + c_k) with a wall one. The
// wall cells' duty of the Table 1 caption (nb_pop_k += pop_kbar towards fluid
// neighbours) is done here by the fluid cell: pop_k(x) += pop_kbar(x - c_k)
// when x - c_k is a wall. Every location is touched by exactly one thread.
template <int Q, class ST, int LAYOUT>
__device__ __forceinline__ void swap_stream_slow(const Field& F, uint32_t i, uint8_t fl)
{
    using S = L<Q>;
    using T = typename ST::T;
    const Acc<ST, LAYOUT, Q, true> a{(T*)F.pop, F.stride};
    const bool border = fl & FL_BORDER;
    const Coord c = border ? cell_coord(i, F) : Coord{0, 0, 0};
    static_for<0, S::half>([&](auto K) {
        constexpr int k = K;
        const uint32_t j = neighbour<Q, k, 1>(F, i, border, c);
        if (is_fluid(F, j)) {
            const T m = *a.ptr(i, S::opp(k));
            const T t = *a.ptr(j, k);
            *a.ptr(i, S::opp(k)) = t;
            *a.ptr(j, k) = m;
        } else {
            a.st(i, S::opp(k), reflect(F, j, a.ld(i, S::opp(k))) + a.ld(j, k));
        }
        const uint32_t s = neighbour<Q, k, -1>(F, i, border, c);
        if (!is_fluid(F, s)) a.st(i, k, reflect(F, s, a.ld(i, k)) + a.ld(s, S::opp(k)));
    });
}

template <int Q, class ST, int LAYOUT, int PART>
__device__ __forceinline__ void cell_swap_stream(const Field& F, uint32_t i)
{
    using S = L<Q>;
    using T = typename ST::T;
    const Acc<ST, LAYOUT, Q, true> a{(T*)F.pop, F.stride};
    const uint8_t fl = F.flags[i];
    if constexpr (PART == PART_SLOW) {
        swap_stream_slow<Q, ST, LAYOUT>(F, i, fl);
    } else {
        T mine[S::half], theirs[S::half];
        static_for<0, S::half>([&](auto K) {
            constexpr int k = K;
            mine[k] = a.raw_ld(i, S::opp(k));
            theirs[k] = a.raw_ld_fast(i, k, offset<Q, k, 1>(F), F.ntot);
        });
        issue_all(mine);
        issue_all(theirs);
        if ((fl & FL_TYPE) != FL_FLUID) return;
        if (!(fl & FL_SLOW)) {
            static_for<0, S::half>([&](auto K) {
                constexpr int k = K;
                if (!wall_to<Q, k>(fl)) {
                    a.raw_st(i, S::opp(k), theirs[k]);
                    a.raw_st_shift(i, k, offset<Q, k, 1>(F), mine[k]);
                } else {  // pop_kbar(x) += pop_k(x + c_k), the wall's term
                    a.st(i, S::opp(k), real_t<ST>(mine[k]) + real_t<ST>(theirs[k]));
                }
                if (wall_from<Q, k>(fl))  // the wall's duty: pop_k(x) += pop_kbar(x - c_k)
                    a.st(i, k, a.ld(i, k) + real_t<ST>(a.raw_ld_shift(i, S::opp(k), offset<Q, k, -1>(F))));
            });
        } else if constexpr (PART == PART_ALL) {
            swap_stream_slow<Q, ST, LAYOUT>(F, i, fl);
        }
    }
}

// AA-pattern, even step (Table 1, row AA/Even): purely local,
// pop_kbar(x) <- f_out_k.
template <int Q, int MODEL, class ST, int LAYOUT>
__device__ __forceinline__ void cell_aa_even(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    cell_swap_collide<Q, MODEL, ST, LAYOUT>(F, p, i);
}

// AA-pattern, odd step (Table 1, row AA/Odd). Pull: f_k(x) is at
// pop_kbar(x - c_k), or pop_k(x) + pop_kbar(x - c_k) across a wall. Collide.
// Push: pop_k(x + c_k) <- f_out_k, or pop_kbar(x) <- f_out_k + pop_k(x + c_k)
// across a wall. A cell writes exactly the locations it read.
template <int Q, int MODEL, class ST, int LAYOUT>
__device__ __forceinline__ void aa_odd_slow(const Field& F, const Relax<real_t<ST>>& p, uint32_t i, uint8_t fl)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> a{(typename ST::T*)F.pop, F.stride};
    const bool border = fl & FL_BORDER;
    const Coord c = border ? cell_coord(i, F) : Coord{0, 0, 0};
    R g[Q];
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == S::rest) {
            g[k] = a.ld(i, k);
        } else {
            const uint32_t s = neighbour<Q, k, -1>(F, i, border, c);
            if (is_fluid(F, s)) g[k] = a.ld(s, S::opp(k));
            else g[k] = reflect(F, s, a.ld(i, k)) + a.ld(s, S::opp(k));
        }
    });
    collide<Q, MODEL, ST::shifted>(g, p);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == S::rest) {
            a.st(i, k, g[k]);
        } else {
            const uint32_t j = neighbour<Q, k, 1>(F, i, border, c);
            if (is_fluid(F, j)) a.st(j, k, g[k]);
            else a.st(i, S::opp(k), reflect(F, j, g[k]) + a.ld(j, k));
        }
    });
}

template <int Q, int MODEL, class ST, int LAYOUT, int PART, bool ZWRAP>
__device__ __forceinline__ void cell_aa_odd(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> a{(typename ST::T*)F.pop, F.stride};
    const uint8_t fl = F.flags[i];
    if constexpr (PART == PART_SLOW) {
        aa_odd_slow<Q, MODEL, ST, LAYOUT>(F, p, i, fl);
    } else {
        if constexpr (PART == PART_ALL) {
            if ((fl & FL_TYPE) == FL_FLUID && (fl & FL_SLOW)) {
                aa_odd_slow<Q, MODEL, ST, LAYOUT>(F, p, i, fl);
                return;
            }
        }
        // ZWRAP variant: z-face cells of a box that wraps in z reach their
        // wrapped neighbours through a per-lane index correction: +nz at
        // z = 0 (reading z - 1, writing z - 1), -nz at z = nz - 1. FP16
        // otherwise: z-face lanes read their own row (face_rows) and store
        // nothing.
        int32_t zp = 0, zm = 0;
        if constexpr (ZWRAP) {
            if (fl & FL_ZWRAP) {
                if (i % (uint32_t)F.nz == 0) zp = F.nz;
                else zm = -F.nz;
            }
        } else if constexpr (sizeof(typename ST::T) == 2) {
            face_rows(F, i, zp, zm);
        }
        R g[Q];
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k == S::rest) {
                g[k] = a.ld(i, k);
            } else {
                const uint32_t j = S::cz(k) > 0 ? i + zp : (S::cz(k) < 0 ? i + zm : i);
                g[k] = a.ld_fast(j, S::opp(k), offset<Q, k, -1>(F), F.ntot);
            }
        });
        issue_all(g);
        if constexpr (!ZWRAP) zp = zm = 0;  // lanes that store are off the z faces
        if (fl & FL_PLANE) {  // pull across the wall plane: pop_k(x) + pop_kbar(x - c_k)
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                if (wall_from<Q, k>(fl)) g[k] += a.ld(i, k);
            });
        }
        collide<Q, MODEL, ST::shifted>(g, p);
        if ((fl & FL_TYPE) != FL_FLUID) return;
        if ((fl & FL_SLOW) && !(ZWRAP && (fl & FL_ZWRAP))) return;  // written by the slow part
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if (!wall_to<Q, k>(fl)) {
                const uint32_t j = S::cz(k) > 0 ? i + zm : (S::cz(k) < 0 ? i + zp : i);
                a.raw_st_shift(j, k, offset<Q, k, 1>(F), to_storage<ST>(g[k]));
            } else {  // push across the wall plane: pop_kbar(x) <- f_out_k + pop_k(x + c_k)
                const R w = R(a.raw_ld_shift(i, k, offset<Q, k, 1>(F)));
                a.st(i, S::opp(k), g[k] + w);
            }
        });
    }
}

// Two-population scheme in pull form, beside the push form of Table 1
// (row 2Pop). The stored state is post-collision with f_out_k in slot kbar,
// as the AA pattern leaves it after an even step. A step gathers f_k(x) from
// pop_kbar(x - c_k), or pop_k(x) + pop_kbar(x - c_k) across a wall (the AA
// odd-step gather), collides, and stores out_kbar(x) <- f_out_k at the
// cell's own index; the arrays then trade places. The shifted accesses are
// the reads, which cost this memory system less than shifted writes.
template <int Q, int MODEL, class ST, int LAYOUT>
__device__ __forceinline__ void pull_slow(const Field& F, const Relax<real_t<ST>>& p, uint32_t i, uint8_t fl)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> a{(typename ST::T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> o{(typename ST::T*)F.out, F.stride};
    const bool border = fl & FL_BORDER;
    const Coord c = border ? cell_coord(i, F) : Coord{0, 0, 0};
    R g[Q];
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == S::rest) {
            g[k] = a.ld(i, k);
        } else {
            const uint32_t s = neighbour<Q, k, -1>(F, i, border, c);
            if (is_fluid(F, s)) g[k] = a.ld(s, S::opp(k));
            else g[k] = gather_across<Q, k, ST>(F, a, i, s, border, c);
        }
    });
    collide<Q, MODEL, ST::shifted>(g, p);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        o.st(i, S::opp(k), g[k]);
    });
}

template <int Q, int MODEL, class ST, int LAYOUT, int PART, bool ZWRAP>
__device__ __forceinline__ void cell_pull(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q, true> a{(typename ST::T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> o{(typename ST::T*)F.out, F.stride};
    const uint8_t fl = F.flags[i];
    if constexpr (PART == PART_SLOW) {
        pull_slow<Q, MODEL, ST, LAYOUT>(F, p, i, fl);
    } else {
        const bool fluid = (fl & FL_TYPE) == FL_FLUID;
        if constexpr (PART == PART_ALL) {
            if (fluid && (fl & FL_SLOW)) {
                pull_slow<Q, MODEL, ST, LAYOUT>(F, p, i, fl);
                return;
            }
        }
        // ZWRAP variant: z-face cells of a box that wraps in z reach their
        // wrapped neighbours through a per-lane index correction of +nz
        // (z = 0, reading z - 1) or -nz (z = nz - 1, reading z + 1).
        int32_t zp = 0, zm = 0;
        if (ZWRAP && (fl & FL_ZWRAP)) {
            if (i % (uint32_t)F.nz == 0) zp = F.nz;
            else zm = -F.nz;
        }
        R g[Q];
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k == S::rest) {
                g[k] = a.ld(i, k);
            } else {
                const uint32_t j = S::cz(k) > 0 ? i + zp : (S::cz(k) < 0 ? i + zm : i);
                g[k] = a.ld_fast(j, S::opp(k), offset<Q, k, -1>(F), F.ntot);
            }
        });
        issue_all(g);
        if (fl & FL_PLANE) {  // across the wall plane: pop_k(x) + pop_kbar(x - c_k)
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                if (wall_from<Q, k>(fl)) g[k] += a.ld(i, k);
            });
        }
        collide<Q, MODEL, ST::shifted>(g, p);
        if (!fluid) {
            // Wall cells write their terms into the other array, which keeps
            // every store instruction writing whole cache lines. With the
            // built-in geometries the terms follow from the cell type and the
            // lid velocity, as at initialisation, so no reload is needed.
            if (!F.custom_walls) {
                static_for<0, Q>([&](auto K) {
                    constexpr int k = K;
                    g[k] = builtin_wall_term<Q, ST, S::opp(k)>(F, fl & FL_TYPE);
                });
            } else {
                static_for<0, Q>([&](auto K) {
                    constexpr int k = K;
                    g[k] = a.ld(i, S::opp(k));
                });
            }
        } else if ((fl & FL_SLOW) && !(ZWRAP && (fl & FL_ZWRAP))) {
            return;  // written by the slow part
        }
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            o.st(i, S::opp(k), g[k]);
        });
    }
}

// ---------------------------------------------------------------------------
// Box cavities of the built-in geometry, with every decision taken from the
// cell's position instead of its flag byte: a cell is fluid iff
// 1 <= x <= nx-2 (and so for y, z), its neighbour x +- c_k is a wall iff it
// leaves that range, and a wall cell is a lid cell iff it lies in the layer
// z = nz-1. Each direction then costs one load and one store whose address
// is chosen per lane (neighbour slot, or the cell's own slot across a wall)
// and the wall terms come from the lid table, so walls, faces, edges and
// corners all stay on one branch-free path, with no flag traffic and no
// second gather round. Used by the ensemble, whose members are such
// cavities; ntot < 2^24 (exact float quotients below).

// Lid term w_J of the table in the storage type.
template <class ST, int J>
__device__ __forceinline__ real_t<ST> lid_value(const Field& F)
{
    if constexpr (sizeof(typename ST::T) == 8) return F.lid.d[J];
    else return F.lid.f[J];
}

struct BoxPos {
    // lo[a]: coordinate a is 1; hi[a]: it is n_a - 2 (both for n_a = 3);
    // top: the cell lies in the lid layer z = nz - 1.
    bool fluid, top, lo[3], hi[3];
};

// floor(n / d) for n < 2^24 and d >= 1: the float quotient is within one of
// the true one, and one correction step fixes it.
__device__ __forceinline__ uint32_t udiv24(uint32_t n, uint32_t d, float rcp)
{
    uint32_t q = (uint32_t)((float)n * rcp);
    const int32_t r = (int32_t)(n - q * d);
    if (r < 0) --q;
    else if (r >= (int32_t)d) ++q;
    return q;
}

__device__ __forceinline__ BoxPos box_pos(const Field& F, uint32_t i, float rcp_nz, float rcp_ny)
{
    const uint32_t row = udiv24(i, (uint32_t)F.nz, rcp_nz);
    const int z = (int)(i - row * (uint32_t)F.nz);
    const uint32_t x = udiv24(row, (uint32_t)F.ny, rcp_ny);
    const int y = (int)(row - x * (uint32_t)F.ny);
    const int c[3] = {(int)x, y, z}, n[3] = {F.nx, F.ny, F.nz};
    BoxPos p;
    p.fluid = true;
    for (int a = 0; a < 3; ++a) {
        p.fluid = p.fluid && c[a] >= 1 && c[a] <= n[a] - 2;
        p.lo[a] = c[a] == 1;
        p.hi[a] = c[a] == n[a] - 2;
    }
    p.top = z == F.nz - 1;
    return p;
}

// The same for a single lattice of any size (i < 2^32): the quotients from
// the 64-bit reciprocals of nz and ny, exact for every 32-bit index.
__device__ __forceinline__ BoxPos box_pos64(const Field& F, uint32_t i)
{
    const uint32_t row = (uint32_t)__umul64hi((unsigned long long)i, F.zrecip);
    const int z = (int)(i - row * (uint32_t)F.nz);
    const uint32_t x = (uint32_t)__umul64hi((unsigned long long)row, F.yrecip);
    const int y = (int)(row - x * (uint32_t)F.ny);
    const int c[3] = {(int)x, y, z}, n[3] = {F.nx, F.ny, F.nz};
    BoxPos p;
    p.fluid = true;
    for (int a = 0; a < 3; ++a) {
        p.fluid = p.fluid && c[a] >= 1 && c[a] <= n[a] - 2;
        p.lo[a] = c[a] == 1;
        p.hi[a] = c[a] == n[a] - 2;
    }
    p.top = z == F.nz - 1;
    return p;
}

// Fluid cell: x + s*c_k is a wall.
template <int Q, int K, int SIGN>
__device__ __forceinline__ bool box_wall(const BoxPos& p)
{
    bool w = false;
    static_for<0, 3>([&](auto A) {
        constexpr int a = A;
        constexpr int c = SIGN * L<Q>::c(K, a);
        if constexpr (c > 0) w = w || p.hi[a];
        else if constexpr (c < 0) w = w || p.lo[a];
    });
    return w;
}

// Fluid cell whose neighbour x + s*c_k is a wall: the stored term of that
// wall cell in slot J, a lid term iff the wall lies in the layer z = nz - 1.
template <int Q, int K, int SIGN, class ST, int J>
__device__ __forceinline__ real_t<ST> box_wall_term(const Field& F, const BoxPos& p)
{
    if constexpr (SIGN * L<Q>::cz(K) > 0) return p.hi[2] ? lid_value<ST, J>(F) : real_t<ST>(0);
    else return real_t<ST>(0);
}

// Pull and AA odd kinds for the built-in cavity of a single lattice (any
// layout), every decision taken from the cell's position as in the box
// kernels below. A fluid lane gathers pop_kbar(x - c_k), or its own pop_k(x)
// plus the wall's term from the lid table across a wall, with one load per
// direction at an address chosen per lane. Pull: store out_kbar(x); wall
// lanes load nothing and write their terms into the other array. AA odd:
// store pop_k(x + c_k), or pop_kbar(x) <- f_out_k + w_k(x + c_k) across a
// wall; wall lanes do nothing. No flag byte, no second round of loads for
// cells next to a wall, and no edge-cell list (edges and corners take the
// same path). The sums are those of the flag-driven kernels, operand for
// operand.
// The same kinds with every address an unsigned 32-bit byte offset from one
// base held in scalar registers. A lane's choice between its own slot and the
// neighbour's is then one 32-bit select (written as arithmetic: the compiler
// would otherwise branch per direction), where two 64-bit pointers into two
// streams cost a select each and kept the loads from issuing together. Two
// addressings qualify: SoA arrays under 4 GiB (F.soa32; the base is the start
// of the halo before stream 0), and the blocked layout when every row of the
// lattice is one run (F.run_rows: nz equal to the run length), where the
// neighbour x - c_k of a fluid cell (1 <= z <= nz - 2) lies a constant number
// of runs away and at most one lane over within its run, so its index is the
// cell's own plus a constant.
template <int Q>
struct SoaOffsets {
    uint32_t lane, ssz, sz;
    __device__ __forceinline__ uint32_t own(int s) const { return lane + (uint32_t)s * ssz; }
    template <int K, int SIGN>
    __device__ __forceinline__ uint32_t nb(const Field& F, int s) const
    {
        return own(s) + (uint32_t)(offset<Q, K, SIGN>(F) * (int32_t)sz);
    }
};

template <int Q>
struct RunOffsets {
    uint32_t lane, sz;  // lane: byte offset of (cell, slot 0)
    __device__ __forceinline__ uint32_t own(int s) const { return lane + (uint32_t)s * kBlockCells * sz; }
    template <int K, int SIGN>
    __device__ __forceinline__ uint32_t nb(const Field& F, int s) const
    {
        constexpr int cx = SIGN * L<Q>::cx(K), cy = SIGN * L<Q>::cy(K), cz = SIGN * L<Q>::cz(K);
        const int32_t runs = cx * F.ny + cy;  // one run per row
        return own(s) + (uint32_t)((runs * Q * (int32_t)kBlockCells + cz) * (int32_t)sz);
    }
};

template <int Q, int MODEL, class ST, int KIND, class A>
__device__ __forceinline__ void box_step_off(const Field& F, const Relax<real_t<ST>>& rp, const BoxPos& p,
                                             const A& ad, const char* src, char* dst)
{
    using S = L<Q>;
    using R = real_t<ST>;
    using T = typename ST::T;
    constexpr bool pull = KIND == KIND_PULL_BOX;
    auto ld = [&](uint32_t o) -> R { return R(*reinterpret_cast<const T*>(src + o)); };
    auto st = [&](uint32_t o, R v) { *reinterpret_cast<T*>(dst + o) = to_storage<ST>(v); };
    // a if c else b, as arithmetic
    auto pick = [](bool c, uint32_t a, uint32_t b) -> uint32_t { return b ^ ((a ^ b) & (0u - (uint32_t)c)); };
    if (!pull && !p.fluid) return;
    R g[Q];
    static_for<0, Q>([&](auto K) { g[K] = R(0); });
    if (p.fluid) {
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k == S::rest) g[k] = ld(ad.own(k));
            else g[k] = ld(pick(box_wall<Q, k, -1>(p), ad.own(k), ad.template nb<k, -1>(F, S::opp(k))));
        });
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k != S::rest)
                if (box_wall<Q, k, -1>(p)) g[k] += box_wall_term<Q, k, -1, ST, S::opp(k)>(F, p);
        });
    }
    collide<Q, MODEL, ST::shifted>(g, rp);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (pull) {
            const R wv = p.top ? lid_value<ST, S::opp(k)>(F) : R(0);
            st(ad.own(S::opp(k)), p.fluid ? g[k] : wv);
        } else if constexpr (k == S::rest) {
            st(ad.own(k), g[k]);
        } else {
            const bool w = box_wall<Q, k, 1>(p);
            st(pick(w, ad.own(S::opp(k)), ad.template nb<k, 1>(F, k)),
               w ? g[k] + box_wall_term<Q, k, 1, ST, k>(F, p) : g[k]);
        }
    });
}

template <int Q, int MODEL, class ST, int LAYOUT, int KIND>
__device__ __forceinline__ void box_step_cell(const Field& F, const Relax<real_t<ST>>& rp, uint32_t i)
{
    using S = L<Q>;
    using R = real_t<ST>;
    using T = typename ST::T;
    constexpr bool pull = KIND == KIND_PULL_BOX;
    const Acc<ST, LAYOUT, Q, true> a{(T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> o{(T*)(pull ? F.out : F.pop), F.stride};
    const BoxPos p = box_pos64(F, i);
    constexpr uint32_t sz = sizeof(T);
    if constexpr (LAYOUT == LAYOUT_SOA) {
        if (F.soa32) {
            const int64_t h = (int64_t)F.ny * F.nz + F.nz + 1;  // the largest neighbour offset
            const SoaOffsets<Q> ad{(i + (uint32_t)h) * sz, (uint32_t)F.stride * sz, sz};
            box_step_off<Q, MODEL, ST, KIND>(F, rp, p, ad, reinterpret_cast<const char*>(F.pop) - h * sz,
                                             reinterpret_cast<char*>(pull ? F.out : F.pop) - h * sz);
            return;
        }
    } else if constexpr (LAYOUT == LAYOUT_BLOCKED) {
        if (F.run_rows) {
            constexpr uint32_t B = kBlockCells;
            const uint32_t j = i + (uint32_t)F.stride;  // past the halo runs
            const RunOffsets<Q> ad{((j & ~(B - 1)) * (uint32_t)Q + (j & (B - 1))) * sz, sz};
            box_step_off<Q, MODEL, ST, KIND>(F, rp, p, ad, reinterpret_cast<const char*>(F.pop),
                                             reinterpret_cast<char*>(pull ? F.out : F.pop));
            return;
        }
    }
    if (!pull && !p.fluid) return;
    R g[Q];
    static_for<0, Q>([&](auto K) { g[K] = R(0); });
    if (p.fluid) {
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k == S::rest) {
                g[k] = a.ld(i, k);
            } else {
                const T* const own = a.ptr(i, k);
                const T* const nb = a.ptr_shift(i, S::opp(k), offset<Q, k, -1>(F));
                g[k] = R(*(box_wall<Q, k, -1>(p) ? own : nb));
            }
        });
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (k != S::rest)
                if (box_wall<Q, k, -1>(p)) g[k] += box_wall_term<Q, k, -1, ST, S::opp(k)>(F, p);
        });
    }
    collide<Q, MODEL, ST::shifted>(g, rp);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (pull) {
            const R wv = p.top ? lid_value<ST, S::opp(k)>(F) : R(0);  // a wall lane's term in slot kbar
            o.st(i, S::opp(k), p.fluid ? g[k] : wv);
        } else if constexpr (k == S::rest) {
            o.st(i, k, g[k]);
        } else {
            const bool w = box_wall<Q, k, 1>(p);
            T* const dst = w ? o.ptr(i, S::opp(k)) : o.ptr_shift(i, k, offset<Q, k, 1>(F));
            *dst = to_storage<ST>(w ? g[k] + box_wall_term<Q, k, 1, ST, k>(F, p) : g[k]);
        }
    });
}

// The same two kinds for the built-in periodic box (every cell fluid): the
// neighbour index x +- c_k wraps on the faces by a per-lane correction taken
// from the cell's position, so the z-face and the x / y-face cells need
// neither the flag byte nor the edge-cell list. Gather f_k(x) from
// pop_kbar(x - c_k); pull: store out_kbar(x); AA odd: store pop_k(x + c_k).
struct WrapPos {
    uint32_t lo[3], hi[3];  // N_a * span_a on the low / high face of axis a, else 0
};

__device__ __forceinline__ WrapPos wrap_pos(const Field& F, uint32_t i)
{
    // (a reciprocal of 0 stands for an axis of one cell)
    const uint32_t row = F.zrecip ? (uint32_t)__umul64hi((unsigned long long)i, F.zrecip) : i;
    const uint32_t z = i - row * (uint32_t)F.nz;
    const uint32_t x = F.yrecip ? (uint32_t)__umul64hi((unsigned long long)row, F.yrecip) : row;
    const uint32_t y = row - x * (uint32_t)F.ny;
    const uint32_t plane = (uint32_t)F.ny * (uint32_t)F.nz;
    WrapPos w;
    w.lo[0] = x == 0 ? F.ntot : 0u;
    w.hi[0] = x == (uint32_t)F.nx - 1 ? F.ntot : 0u;
    w.lo[1] = y == 0 ? plane : 0u;
    w.hi[1] = y == (uint32_t)F.ny - 1 ? plane : 0u;
    w.lo[2] = z == 0 ? (uint32_t)F.nz : 0u;
    w.hi[2] = z == (uint32_t)F.nz - 1 ? (uint32_t)F.nz : 0u;
    return w;
}

// Index of x + SIGN c_K in the periodic box (32-bit arithmetic: the result
// lies in [0, ntot)).
template <int Q, int K, int SIGN>
__device__ __forceinline__ uint32_t wrap_neighbour(const Field& F, uint32_t i, const WrapPos& w)
{
    uint32_t j = i + (uint32_t)offset<Q, K, SIGN>(F);
    static_for<0, 3>([&](auto A) {
        constexpr int a = A;
        constexpr int c = SIGN * L<Q>::c(K, a);
        if constexpr (c > 0) j -= w.hi[a];
        else if constexpr (c < 0) j += w.lo[a];
    });
    return j;
}

template <int Q, int MODEL, class ST, int LAYOUT, int KIND>
__device__ __forceinline__ void wrap_step_cell(const Field& F, const Relax<real_t<ST>>& rp, uint32_t i)
{
    using S = L<Q>;
    using R = real_t<ST>;
    using T = typename ST::T;
    constexpr bool pull = KIND == KIND_PULL_WRAP;
    const Acc<ST, LAYOUT, Q, true> a{(T*)F.pop, F.stride};
    const Acc<ST, LAYOUT, Q, true> o{(T*)(pull ? F.out : F.pop), F.stride};
    const WrapPos w = wrap_pos(F, i);
    R g[Q];
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == S::rest) g[k] = a.ld(i, k);
        else g[k] = a.ld(wrap_neighbour<Q, k, -1>(F, i, w), S::opp(k));
    });
    collide<Q, MODEL, ST::shifted>(g, rp);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (pull) o.st(i, S::opp(k), g[k]);
        else if constexpr (k == S::rest) o.st(i, k, g[k]);
        else o.st(wrap_neighbour<Q, k, 1>(F, i, w), k, g[k]);
    });
}

template <int Q, int MODEL, class ST, int LAYOUT, int KIND, int PART>
__device__ __forceinline__ void cell_step(const Field& F, const Relax<real_t<ST>>& p, uint32_t i)
{
    if constexpr (KIND == KIND_2POP) cell_2pop<Q, MODEL, ST, LAYOUT, PART>(F, p, i);
    else if constexpr (KIND == KIND_SWAP_COLLIDE) cell_swap_collide<Q, MODEL, ST, LAYOUT>(F, p, i);
    else if constexpr (KIND == KIND_SWAP_STREAM) cell_swap_stream<Q, ST, LAYOUT, PART>(F, i);
    else if constexpr (KIND == KIND_AA_EVEN) cell_aa_even<Q, MODEL, ST, LAYOUT>(F, p, i);
    else if constexpr (KIND == KIND_AA_ODD) cell_aa_odd<Q, MODEL, ST, LAYOUT, PART, false>(F, p, i);
    else if constexpr (KIND == KIND_AA_ODD_Z) cell_aa_odd<Q, MODEL, ST, LAYOUT, PART, true>(F, p, i);
    else if constexpr (KIND == KIND_PULL) cell_pull<Q, MODEL, ST, LAYOUT, PART, false>(F, p, i);
    else if constexpr (KIND == KIND_PULL_Z) cell_pull<Q, MODEL, ST, LAYOUT, PART, true>(F, p, i);
    else if constexpr (KIND == KIND_PULL_BOX || KIND == KIND_AA_ODD_BOX) box_step_cell<Q, MODEL, ST, LAYOUT, KIND>(F, p, i);
    else wrap_step_cell<Q, MODEL, ST, LAYOUT, KIND>(F, p, i);
}

// Block b of nb fast-part blocks in the order the cells are visited.
__device__ __forceinline__ uint32_t step_block(const Field& F, uint32_t b, uint32_t nb)
{
    b = F.reverse ? nb - 1 - b : b;
    if (LBM_XCD_REMAP) {
        const uint32_t per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    return b;
}

// Register budget of the fast step kernels: room for min_step_waves waves
// per SIMD.
#define LBM_STEP_ATTR(Q, ST, KIND) \
    __attribute__((amdgpu_waves_per_eu(min_step_waves(Q, (int)sizeof(typename ST::T), KIND))))

// Kinds whose cells reach their neighbours, and so have an edge-cell part;
// the z-wrap variants of the fast part share the edge part of their kind.
constexpr bool has_edge_part(int kind)
{
    return kind == KIND_2POP || kind == KIND_SWAP_STREAM || kind == KIND_AA_ODD || kind == KIND_PULL ||
           kind == KIND_PULL_Z || kind == KIND_AA_ODD_Z;
}

constexpr int edge_kind(int kind)
{
    return kind == KIND_PULL_Z ? KIND_PULL : (kind == KIND_AA_ODD_Z ? KIND_AA_ODD : kind);
}

// One launch per step: the first edge_blocks blocks take the cells of the
// edge-cell list (the edge part), the others every cell of the lattice (the
// fast part, which leaves the listed cells alone). The two parts touch
// disjoint memory, since every cell owns the locations it reads and writes,
// so they need no order between them; the listed cells come first, so that
// their scattered, latency-bound accesses overlap the streaming of the fast
// part and the step needs no second stream.
template <int Q, int MODEL, class ST, int LAYOUT, int KIND>
__global__ void __launch_bounds__(max_step_block(Q, MODEL, (int)sizeof(typename ST::T))) LBM_STEP_ATTR(Q, ST, KIND)
    k_step(Field F, RelaxD pd, const uint32_t* __restrict__ list, uint32_t n_edge, uint32_t edge_blocks)
{
    if constexpr (has_edge_part(KIND)) {
        if (blockIdx.x < edge_blocks) {
            const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
            if (j >= n_edge) return;
            const uint32_t i = list[F.reverse ? n_edge - 1 - j : j];
            if (i >= F.ntot) return;
            cell_step<Q, MODEL, ST, LAYOUT, edge_kind(KIND), PART_SLOW>(F, relax_of<real_t<ST>>(pd), i);
            return;
        }
    }
    const uint32_t i = step_block(F, blockIdx.x - edge_blocks, gridDim.x - edge_blocks) * blockDim.x + threadIdx.x;
    if (i >= F.ntot) return;
    cell_step<Q, MODEL, ST, LAYOUT, KIND, PART_FAST>(F, relax_of<real_t<ST>>(pd), i);
}

// ---------------------------------------------------------------------------
// Fast part with CPT consecutive cells per lane (SoA): every stream access is
// one CPT-wide vector (aligned to the element, not the vector, since
// neighbour shifts move it by one element).
template <class T, int N>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(N), aligned(sizeof(T))));
};

template <int CPT>
__device__ __forceinline__ bool group_fast(const uint8_t* flags, uint32_t i0)
{
    if constexpr (CPT == 2) return (*reinterpret_cast<const uint16_t*>(flags + i0) & 0xDFDFu) == 0;
    else if constexpr (CPT == 4) return (*reinterpret_cast<const uint32_t*>(flags + i0) & 0xDFDFDFDFu) == 0;
    else if constexpr (CPT == 8) return (*reinterpret_cast<const uint64_t*>(flags + i0) & 0xDFDFDFDFDFDFDFDFull) == 0;
    else return (flags[i0] & (FL_TYPE | FL_SLOW | FL_PLANE)) == FL_FLUID;
}

template <int Q, int MODEL, class ST, int KIND, int CPT>
__device__ __forceinline__ void group_step(const Field& F, const Relax<real_t<ST>>& p, uint32_t i0)
{
    using S = L<Q>;
    using R = real_t<ST>;
    using T = typename ST::T;
    using V = typename VecOf<T, CPT>::type;
    const Acc<ST, LAYOUT_SOA, Q, true> a{(T*)F.pop, F.stride};
    const Acc<ST, LAYOUT_SOA, Q, true> o{(T*)(KIND == KIND_2POP ? F.out : F.pop), F.stride};
    const bool fast = group_fast<CPT>(F.flags, i0);
    if constexpr (KIND == KIND_SWAP_STREAM) {
        V mine[S::half], theirs[S::half];
        static_for<0, S::half>([&](auto K) {
            constexpr int k = K;
            mine[k] = *reinterpret_cast<const V*>(a.ptr(i0, S::opp(k)));
            theirs[k] = *reinterpret_cast<const V*>(a.ptr_shift(i0, k, offset<Q, k, 1>(F)));
        });
        issue_all(mine);
        issue_all(theirs);
        if (!fast) return;
        static_for<0, S::half>([&](auto K) {
            constexpr int k = K;
            *reinterpret_cast<V*>(a.ptr(i0, S::opp(k))) = theirs[k];
            *reinterpret_cast<V*>(a.ptr_shift(i0, k, offset<Q, k, 1>(F))) = mine[k];
        });
    } else {
        V v[Q];
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (KIND == KIND_AA_ODD && k != S::rest)
                v[k] = *reinterpret_cast<const V*>(a.ptr_shift(i0, S::opp(k), offset<Q, k, -1>(F)));
            else
                v[k] = *reinterpret_cast<const V*>(a.ptr(i0, k));
        });
        issue_all(v);
        V w[Q];
        static_for<0, CPT>([&](auto C) {
            constexpr int c = C;
            R g[Q];
            static_for<0, Q>([&](auto K) { g[K] = R(v[K][c]); });
            collide<Q, MODEL, ST::shifted>(g, p);
            static_for<0, Q>([&](auto K) { w[K][c] = to_storage<ST>(g[K]); });
        });
        if (!fast) return;
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (KIND == KIND_AA_EVEN || KIND == KIND_SWAP_COLLIDE)
                *reinterpret_cast<V*>(o.ptr(i0, S::opp(k))) = w[k];
            else
                *reinterpret_cast<V*>(o.ptr_shift(i0, k, offset<Q, k, 1>(F))) = w[k];
        });
    }
}

template <int Q, int MODEL, class ST, int KIND, int CPT>
__global__ void __launch_bounds__(256) LBM_STEP_ATTR(Q, ST, KIND) k_step_vec(Field F, RelaxD pd)
{
    const uint32_t i0 = (step_block(F, blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) * CPT;
    if (i0 + CPT > F.ntot) return;  // a ragged tail is in the near-wall list
    group_step<Q, MODEL, ST, KIND, CPT>(F, relax_of<real_t<ST>>(pd), i0);
}

// Fast and slow parts in one pass over every cell (one launch per step, as
// the per-cavity reference path of the batched ensemble uses).
template <int Q, int MODEL, class ST, int LAYOUT, int KIND>
__global__ void __launch_bounds__(max_step_block(Q, MODEL, (int)sizeof(typename ST::T))) LBM_STEP_ATTR(Q, ST, KIND) k_step_all(Field F, RelaxD pd)
{
    const uint32_t i = step_block(F, blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= F.ntot) return;
    cell_step<Q, MODEL, ST, LAYOUT, KIND, PART_ALL>(F, relax_of<real_t<ST>>(pd), i);
}

// Slow part over the listed cells (fluid cells next to a wall or on a
// periodic face); only the kinds that touch neighbours have one.
template <int Q, int MODEL, class ST, int LAYOUT, int KIND>
__global__ void __launch_bounds__(256) k_step_slow(Field F, RelaxD pd, const uint32_t* __restrict__ list, uint32_t n)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = list[F.reverse ? n - 1 - j : j];
    if (i >= F.ntot) return;
    cell_step<Q, MODEL, ST, LAYOUT, KIND, PART_SLOW>(F, relax_of<real_t<ST>>(pd), i);
}

// One step of one cell of a box cavity. AA even: local collide, slot kbar.
// AA odd: gather f_k from pop_kbar(x - c_k), or pop_k(x) + w_kbar(x - c_k)
// across a wall; collide; push f_out_k to pop_k(x + c_k), or pop_kbar(x) <-
// f_out_k + w_k(x + c_k) across a wall (Table 1, row AA). Pull: the same
// gather from pop, then out_kbar(x) <- f_out_k. Every fluid lane runs the
// same instructions: one load and one store per direction, each at a byte
// offset from the array base chosen per lane. Wall lanes load nothing; in
// the pull kind they write their own terms into out, which keeps its lines
// written whole (measured on the ensemble: pull 30.9 k MLUPS with these
// stores, 19.7 k without), while the AA kinds run faster without them
// (29.7 k against 28.9 k). The sums are the ones the flag-driven kernels
// form, operand for operand, so the results are the same bits.
template <int Q, int MODEL, class ST, int KIND>
__device__ __forceinline__ void box_cell(const Field& F, const Relax<real_t<ST>>& rp, uint32_t i, const BoxPos& p)
{
    using S = L<Q>;
    using R = real_t<ST>;
    using T = typename ST::T;
    constexpr uint32_t sz = sizeof(T);
    char* const src = (char*)F.pop;
    char* const dst = (char*)(KIND == KIND_PULL ? F.out : F.pop);
    const uint32_t sb = (uint32_t)F.stride * sz;  // bytes between streams (< 2^32 / Q here)
    const uint32_t ib = i * sz;
    auto at = [&](char* base, uint32_t off) -> T* { return reinterpret_cast<T*>(base + off); };
    if (KIND != KIND_PULL && !p.fluid) return;
    R g[Q];
    static_for<0, Q>([&](auto K) { g[K] = R(0); });
    if (p.fluid) {
        static_for<0, Q>([&](auto K) {
            constexpr int k = K;
            if constexpr (KIND == KIND_AA_EVEN || k == S::rest) {
                g[k] = R(*at(src, k * sb + ib));
            } else {  // pop_kbar(x - c_k), or pop_k(x) across a wall
                const uint32_t nb = S::opp(k) * sb + ib + (uint32_t)(offset<Q, k, -1>(F) * (int32_t)sz);
                g[k] = R(*at(src, box_wall<Q, k, -1>(p) ? k * sb + ib : nb));
            }
        });
        if constexpr (KIND != KIND_AA_EVEN) {
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                if constexpr (k != S::rest)
                    if (box_wall<Q, k, -1>(p)) g[k] += box_wall_term<Q, k, -1, ST, S::opp(k)>(F, p);
            });
        }
    }
    collide<Q, MODEL, ST::shifted>(g, rp);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        const R wv = p.top ? lid_value<ST, S::opp(k)>(F) : R(0);  // a wall lane's term in slot kbar
        if constexpr (KIND == KIND_AA_EVEN || KIND == KIND_PULL) {
            *at(dst, S::opp(k) * sb + ib) = to_storage<ST>(p.fluid ? g[k] : wv);
        } else if constexpr (k == S::rest) {
            *at(dst, k * sb + ib) = to_storage<ST>(p.fluid ? g[k] : wv);
        } else {
            // Fluid: pop_k(x + c_k) <- f_out_k, or pop_kbar(x) <- f_out_k +
            // w_k(x + c_k) across a wall. Wall lane: its own slot kbar.
            const bool w = box_wall<Q, k, 1>(p);
            const uint32_t nb = k * sb + ib + (uint32_t)(offset<Q, k, 1>(F) * (int32_t)sz);
            const uint32_t off = p.fluid && !w ? nb : S::opp(k) * sb + ib;
            const R v = !p.fluid ? wv : (w ? g[k] + box_wall_term<Q, k, 1, ST, k>(F, p) : g[k]);
            *at(dst, off) = to_storage<ST>(v);
        }
    });
}

// ---------------------------------------------------------------------------
// Batched ensemble, fast part: one launch over a table of (cavity, tile)
// entries, one block per entry. A tile is `cpt` consecutive runs of
// blockDim cells of one cavity, counted from the first cell of the layer
// x = 1: the layers x = 0 and x = nx - 1 are walls that no step needs to
// touch (their slots are whole runs of cache lines, so leaving them alone
// costs no partial-line writes). Fluid cells next to two or more walls
// (edges and corners) are left to the edge-cell kernel below; wall lanes
// write their terms back.
template <int Q, int MODEL, class ST, int KIND>
__global__ void __launch_bounds__(max_step_block(Q, MODEL, (int)sizeof(typename ST::T)))
    LBM_STEP_ATTR(Q, ST, KIND) k_step_batch(const BatchCavity* __restrict__ cav, const uint32_t* __restrict__ tiles,
                                            uint32_t cpt, uint32_t xcd)
{
    const uint32_t b = xcd ? (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const uint32_t t = tiles[b];
    if (t == 0xffffffffu) return;  // padding of the table to a multiple of eight
    const BatchCavity& B = cav[t >> 16];
    const uint32_t plane = (uint32_t)B.F.ny * (uint32_t)B.F.nz;
    const uint32_t end = B.F.ntot - plane;
    uint32_t i = plane + (t & 0xffffu) * blockDim.x * cpt + threadIdx.x;
    const Relax<real_t<ST>> p = relax_of<real_t<ST>>(B.relax);
    for (uint32_t r = 0; r < cpt && i < end; ++r, i += blockDim.x)
        cell_step<Q, MODEL, ST, LAYOUT_SOA, KIND, PART_FAST>(B.F, p, i);
}

// Batched ensemble of box cavities, every cell on the position-driven path
// (AA and pull kinds; cavities of fewer than 2^24 cells): the same tiles as
// above, no edge-cell kernel.
template <int Q, int MODEL, class ST, int KIND>
__global__ void __launch_bounds__(max_step_block(Q, MODEL, (int)sizeof(typename ST::T)))
    LBM_STEP_ATTR(Q, ST, KIND) k_step_batch_box(const BatchCavity* __restrict__ cav,
                                                const uint32_t* __restrict__ tiles, uint32_t cpt, uint32_t xcd)
{
    // xcd: the table is dealt in eight contiguous parts, one per XCD (blocks
    // go to the XCDs in turn), so that the tiles of one cavity, and the
    // neighbours they share, stay in one XCD's L2.
    const uint32_t b = xcd ? (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const uint32_t t = tiles[b];
    if (t == 0xffffffffu) return;  // padding of the table to a multiple of eight
    const BatchCavity& B = cav[t >> 16];
    const uint32_t plane = (uint32_t)B.F.ny * (uint32_t)B.F.nz;
    const uint32_t end = B.F.ntot - plane;
    uint32_t i = plane + (t & 0xffffu) * blockDim.x * cpt + threadIdx.x;
    const float rz = 1.0f / (float)B.F.nz, ry = 1.0f / (float)B.F.ny;
    const Relax<real_t<ST>> p = relax_of<real_t<ST>>(B.relax);
    for (uint32_t r = 0; r < cpt && i < end; ++r, i += blockDim.x)
        box_cell<Q, MODEL, ST, KIND>(B.F, p, i, box_pos(B.F, i, rz, ry));
}

// Batched ensemble, edge part: the listed fluid cells off the fast path,
// grouped by cavity so that each wave of 64 entries belongs to one cavity
// (wave_cav; unused entries hold 0xffffffff), which keeps the cavity's
// description in scalar registers.
template <int Q, int MODEL, class ST, int KIND>
__global__ void __launch_bounds__(256) k_step_batch_slow(const BatchCavity* __restrict__ cav,
                                                        const uint32_t* __restrict__ wave_cav,
                                                        const uint32_t* __restrict__ list, uint32_t n)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    // Every lane of a wave holds the same j >> 6.
    const uint32_t c = __builtin_amdgcn_readfirstlane(wave_cav[j >> 6]);
    const uint32_t i = list[j];
    const BatchCavity& B = cav[c];
    if (i >= B.F.ntot) return;
    cell_step<Q, MODEL, ST, LAYOUT_SOA, KIND, PART_SLOW>(B.F, relax_of<real_t<ST>>(B.relax), i);
}

// ---------------------------------------------------------------------------
// Read-outs. Natural pre-collision populations of one cell (FP64): after an
// AA even step the odd-step pull is applied without collision; shifted
// storage is decoded as f = g + t_k; wall cells return their stored terms.
template <int Q, class ST, int LAYOUT>
__device__ __forceinline__ void natural_cell(const Field& F, uint32_t i, int aa_odd, double (&f)[Q])
{
    using S = L<Q>;
    using R = real_t<ST>;
    const Acc<ST, LAYOUT, Q> a{(typename ST::T*)F.pop, F.stride};
    const uint8_t fl = F.flags[i];
    if ((fl & FL_TYPE) != FL_FLUID) {
        // a pressure wall's term is stored less 2 t_k in shifted storage
        const bool p = ST::shifted && (fl & FL_TYPE) == FL_PRESSURE;
        static_for<0, Q>([&](auto K) { f[K] = double(a.ld(i, K)) + (p ? 2.0 * S::t(K) : 0.0); });
        return;
    }
    const bool border = fl & FL_BORDER;
    const Coord c = border ? cell_coord(i, F) : Coord{0, 0, 0};
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        R v;
        if (!aa_odd || k == S::rest) {
            v = a.ld(i, k);
        } else {
            const uint32_t s = neighbour<Q, k, -1>(F, i, border, c);
            if (is_fluid(F, s)) v = a.ld(s, S::opp(k));
            else v = gather_across<Q, k, ST>(F, a, i, s, border, c);
        }
        f[k] = ST::shifted ? double(v) + S::t(k) : double(v);
    });
}

template <int Q, class ST, int LAYOUT>
__global__ void k_get_populations(Field F, int aa_odd, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.ntot) return;
    double f[Q];
    natural_cell<Q, ST, LAYOUT>(F, i, aa_odd, f);
    static_for<0, Q>([&](auto K) { out[(size_t)K * F.ntot + i] = f[K]; });
}

template <int Q, class ST, int LAYOUT>
__global__ void k_get_cells(Field F, int aa_odd, const int64_t* __restrict__ cells, int n, double* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t c = cells[j];
    if (c < 0 || c >= (int64_t)F.ntot) return;
    double f[Q];
    natural_cell<Q, ST, LAYOUT>(F, (uint32_t)c, aa_odd, f);
    static_for<0, Q>([&](auto K) { out[(size_t)j * Q + K] = f[K]; });
}

template <int Q>
__device__ __forceinline__ void density_velocity(const double (&f)[Q], double& rho, double (&u)[3])
{
    using S = L<Q>;
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        r += f[k];
        static_for<0, 3>([&](auto D) {
            constexpr int a = D;
            if constexpr (S::c(k, a) == 1) j[a] += f[k];
            else if constexpr (S::c(k, a) == -1) j[a] -= f[k];
        });
    });
    rho = r;
    u[0] = j[0] / r;
    u[1] = j[1] / r;
    u[2] = j[2] / r;
}

template <int Q, class ST, int LAYOUT>
__global__ void k_macroscopic(Field F, int aa_odd, double* __restrict__ rho, double* __restrict__ u)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.ntot) return;
    if ((F.flags[i] & FL_TYPE) != FL_FLUID) {
        rho[i] = 0.0;
        u[i] = u[(size_t)F.ntot + i] = u[2 * (size_t)F.ntot + i] = 0.0;
        return;
    }
    double f[Q], r, v[3];
    natural_cell<Q, ST, LAYOUT>(F, i, aa_odd, f);
    density_velocity<Q>(f, r, v);
    rho[i] = r;
    u[i] = v[0];
    u[(size_t)F.ntot + i] = v[1];
    u[2 * (size_t)F.ntot + i] = v[2];
}

// Load natural populations into fluid cells (natural slots, AA phase even).
template <int Q, class ST, int LAYOUT>
__global__ void k_set_populations(Field F, const double* __restrict__ f)
{
    using S = L<Q>;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.ntot || (F.flags[i] & FL_TYPE) != FL_FLUID) return;
    const Acc<ST, LAYOUT, Q> a{(typename ST::T*)F.pop, F.stride};
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        const double v = f[(size_t)k * F.ntot + i];
        a.st(i, k, real_t<ST>(ST::shifted ? v - S::t(k) : v));
    });
}

// Fluid cells: the model's equilibrium at (rho, u) (rho = 1, u = 0 when the
// pointers are null). Wall cells: the momentum-exchange terms of Eq. storage2,
// -6 t_k rho_w c_k . u_w, from the per-cell wall velocity and density when
// given, else from the lid velocity on lid cells (rho_w = 1); with keep_walls
// they keep what they store. Written to pop and, if not null, to out.
template <int Q, int MODEL, class ST, int LAYOUT>
__global__ void k_init(Field F, InitArgs ia)
{
    using R = real_t<ST>;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.ntot) return;
    const uint8_t type = F.flags[i] & FL_TYPE;
    R g[Q];
    if (type != FL_FLUID) {
        if (ia.keep_walls) return;
        if (type == FL_PRESSURE) {
            // 2 t_k rho_w [1 + 9/2 (c_k . u_w)^2 - 3/2 |u_w|^2]. Shifted
            // storage keeps the reflection g_k = -g_out_kbar + stored in
            // shifted values (f = g + t_k on both sides) by storing the term
            // less 2 t_k, formed as 2 t_k (rho_w [...] - 1).
            const double rw = ia.wall_rho ? ia.wall_rho[i] : 1.0;
            double uw[3] = {0.0, 0.0, 0.0};
            if (ia.wall_u) {
                uw[0] = ia.wall_u[i];
                uw[1] = ia.wall_u[(size_t)F.ntot + i];
                uw[2] = ia.wall_u[2 * (size_t)F.ntot + i];
            }
            const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                const double cu = L<Q>::cx(k) * uw[0] + L<Q>::cy(k) * uw[1] + L<Q>::cz(k) * uw[2];
                const double e = rw * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                g[k] = R(2.0 * L<Q>::t(k) * (ST::shifted ? e - 1.0 : e));
            });
        } else if (ia.wall_u || ia.wall_rho) {
            const double rw = ia.wall_rho ? ia.wall_rho[i] : 1.0;
            double uw[3] = {0.0, 0.0, 0.0};
            if (ia.wall_u) {
                uw[0] = ia.wall_u[i];
                uw[1] = ia.wall_u[(size_t)F.ntot + i];
                uw[2] = ia.wall_u[2 * (size_t)F.ntot + i];
            }
            static_for<0, Q>([&](auto K) {
                constexpr int k = K;
                const double cu = L<Q>::cx(k) * uw[0] + L<Q>::cy(k) * uw[1] + L<Q>::cz(k) * uw[2];
                g[k] = R(-6.0 * L<Q>::t(k) * rw * cu);
            });
        } else {
            static_for<0, Q>([&](auto K) { g[K] = builtin_wall_term<Q, ST, K>(F, type); });
        }
    } else {
        const R rho = ia.rho ? R(ia.rho[i]) : R(1);
        R u[3] = {R(0), R(0), R(0)};
        if (ia.u) {
            u[0] = R(ia.u[i]);
            u[1] = R(ia.u[(size_t)F.ntot + i]);
            u[2] = R(ia.u[2 * (size_t)F.ntot + i]);
        }
        equilibrium<Q, MODEL, ST::shifted>(rho, u, g);
    }
    const Acc<ST, LAYOUT, Q> a{(typename ST::T*)F.pop, F.stride};
    static_for<0, Q>([&](auto K) { a.st(i, K, g[K]); });
    if (F.out) {
        const Acc<ST, LAYOUT, Q> b{(typename ST::T*)F.out, F.stride};
        static_for<0, Q>([&](auto K) { b.st(i, K, g[K]); });
    }
}

// Global FP64 mass and kinetic energy: each block reduces its cells
// (wavefront shuffles, then LDS) and writes one partial pair; a second
// single-block pass sums the partials in index order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int Q, class ST, int LAYOUT>
__global__ void __launch_bounds__(256) k_invariants(Field F, int aa_odd, double* __restrict__ partial)
{
    __shared__ double sm[2][4];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double mass = 0.0, ke = 0.0;
    if (i < F.ntot && (F.flags[i] & FL_TYPE) == FL_FLUID) {
        double f[Q], r, v[3];
        natural_cell<Q, ST, LAYOUT>(F, i, aa_odd, f);
        density_velocity<Q>(f, r, v);
        static_for<0, Q>([&](auto K) { mass += f[K]; });
        ke = 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    mass = wave_sum(mass);
    ke = wave_sum(ke);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sm[0][w] = mass;
        sm[1][w] = ke;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, e = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            m += sm[0][k];
            e += sm[1][k];
        }
        partial[2 * (size_t)blockIdx.x] = m;
        partial[2 * (size_t)blockIdx.x + 1] = e;
    }
}

template <int Q>
__global__ void k_neighbors(Field F, const int64_t* __restrict__ cells, int n, int64_t* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (cells[j] < 0 || cells[j] >= (int64_t)F.ntot) {
        for (int k = 0; k < Q; ++k) out[(size_t)j * Q + k] = -1;
        return;
    }
    const uint32_t i = (uint32_t)cells[j];
    const bool border = F.flags[i] & FL_BORDER;
    const Coord c = cell_coord(i, F);
    static_for<0, Q>([&](auto K) {
        constexpr int k = K;
        uint32_t nb;
        if (border || (F.flags[i] & FL_TYPE) != FL_FLUID) {
            nb = neighbour<Q, k, 1>(F, i, true, c);
        } else {
            nb = (uint32_t)((int32_t)i + offset<Q, k, 1>(F));
        }
        out[(size_t)j * Q + k] = nb;
    });
}

}  // namespace lbm
