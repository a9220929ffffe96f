// Launch dispatcher of one (Q, storage) kernel translation unit: maps the
// runtime model / layout / kind of a Launch onto kernel instantiations.
#pragma once

#include "kernels.hpp"

namespace lbm {

template <int Q, int MODEL, class ST, int LAYOUT>
hipError_t launch_step_kind(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(L.block);
    constexpr int CPT = cells_per_thread((int)sizeof(typename ST::T));
    if constexpr (CPT > 1 && LAYOUT == LAYOUT_SOA) {
        switch (L.kind) {
        case KIND_2POP: k_step_vec<Q, MODEL, ST, KIND_2POP, CPT><<<g, b, 0, s>>>(L.F, L.relax); break;
        case KIND_SWAP_COLLIDE: k_step_vec<Q, MODEL, ST, KIND_SWAP_COLLIDE, CPT><<<g, b, 0, s>>>(L.F, L.relax); break;
        case KIND_SWAP_STREAM: k_step_vec<Q, BGK, ST, KIND_SWAP_STREAM, CPT><<<g, b, 0, s>>>(L.F, L.relax); break;
        case KIND_AA_EVEN: k_step_vec<Q, MODEL, ST, KIND_AA_EVEN, CPT><<<g, b, 0, s>>>(L.F, L.relax); break;
        case KIND_AA_ODD: k_step_vec<Q, MODEL, ST, KIND_AA_ODD, CPT><<<g, b, 0, s>>>(L.F, L.relax); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const uint32_t lds = L.lds;
    // edge part in the first L.edge_blocks blocks (kinds that have one)
    const uint32_t* const el = L.slow_list;
    const uint32_t ne = L.n_slow, eb = L.edge_blocks;
    switch (L.kind) {
    case KIND_2POP: k_step<Q, MODEL, ST, LAYOUT, KIND_2POP><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_SWAP_COLLIDE:
        k_step<Q, MODEL, ST, LAYOUT, KIND_SWAP_COLLIDE><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0);
        break;
    case KIND_SWAP_STREAM: k_step<Q, BGK, ST, LAYOUT, KIND_SWAP_STREAM><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_AA_EVEN: k_step<Q, MODEL, ST, LAYOUT, KIND_AA_EVEN><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0); break;
    case KIND_AA_ODD: k_step<Q, MODEL, ST, LAYOUT, KIND_AA_ODD><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_PULL: k_step<Q, MODEL, ST, LAYOUT, KIND_PULL><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_PULL_Z: k_step<Q, MODEL, ST, LAYOUT, KIND_PULL_Z><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_AA_ODD_Z: k_step<Q, MODEL, ST, LAYOUT, KIND_AA_ODD_Z><<<g, b, lds, s>>>(L.F, L.relax, el, ne, eb); break;
    case KIND_PULL_BOX: k_step<Q, MODEL, ST, LAYOUT, KIND_PULL_BOX><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0); break;
    case KIND_AA_ODD_BOX:
        k_step<Q, MODEL, ST, LAYOUT, KIND_AA_ODD_BOX><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0);
        break;
    case KIND_PULL_WRAP:
        k_step<Q, MODEL, ST, LAYOUT, KIND_PULL_WRAP><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0);
        break;
    case KIND_AA_ODD_WRAP:
        k_step<Q, MODEL, ST, LAYOUT, KIND_AA_ODD_WRAP><<<g, b, lds, s>>>(L.F, L.relax, nullptr, 0, 0);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q, int MODEL, class ST, int LAYOUT>
hipError_t launch_all_kind(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(L.block);
    switch (L.kind) {
    case KIND_2POP: k_step_all<Q, MODEL, ST, LAYOUT, KIND_2POP><<<g, b, 0, s>>>(L.F, L.relax); break;
    case KIND_AA_EVEN: k_step_all<Q, MODEL, ST, LAYOUT, KIND_AA_EVEN><<<g, b, 0, s>>>(L.F, L.relax); break;
    case KIND_AA_ODD: k_step_all<Q, MODEL, ST, LAYOUT, KIND_AA_ODD><<<g, b, 0, s>>>(L.F, L.relax); break;
    case KIND_PULL: k_step_all<Q, MODEL, ST, LAYOUT, KIND_PULL><<<g, b, 0, s>>>(L.F, L.relax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q, int MODEL, class ST, int LAYOUT>
hipError_t launch_slow_kind(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(L.block);
    switch (L.kind) {
    case KIND_2POP: k_step_slow<Q, MODEL, ST, LAYOUT, KIND_2POP><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow); break;
    case KIND_SWAP_STREAM:
        k_step_slow<Q, BGK, ST, LAYOUT, KIND_SWAP_STREAM><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow);
        break;
    case KIND_AA_ODD: k_step_slow<Q, MODEL, ST, LAYOUT, KIND_AA_ODD><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow); break;
    case KIND_AA_EVEN: k_step_slow<Q, MODEL, ST, LAYOUT, KIND_AA_EVEN><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow); break;
    case KIND_PULL: k_step_slow<Q, MODEL, ST, LAYOUT, KIND_PULL><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow); break;
    case KIND_SWAP_COLLIDE:
        k_step_slow<Q, MODEL, ST, LAYOUT, KIND_SWAP_COLLIDE><<<g, b, 0, s>>>(L.F, L.relax, L.slow_list, L.n_slow);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q, int MODEL, class ST>
hipError_t launch_batch_kind(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(L.block);
    const uint32_t lds = L.lds;
    if (L.box) {
        switch (L.kind) {
        case KIND_AA_EVEN: k_step_batch_box<Q, MODEL, ST, KIND_AA_EVEN><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
        case KIND_AA_ODD: k_step_batch_box<Q, MODEL, ST, KIND_AA_ODD><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
        case KIND_PULL: k_step_batch_box<Q, MODEL, ST, KIND_PULL><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (L.kind) {
    case KIND_2POP: k_step_batch<Q, MODEL, ST, KIND_2POP><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
    case KIND_AA_EVEN: k_step_batch<Q, MODEL, ST, KIND_AA_EVEN><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
    case KIND_AA_ODD: k_step_batch<Q, MODEL, ST, KIND_AA_ODD><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
    case KIND_PULL: k_step_batch<Q, MODEL, ST, KIND_PULL><<<g, b, lds, s>>>(L.cav, L.tiles, L.cpt, L.xcd); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q, int MODEL, class ST>
hipError_t launch_batch_slow_kind(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(256);
    switch (L.kind) {
    case KIND_2POP:
        k_step_batch_slow<Q, MODEL, ST, KIND_2POP><<<g, b, 0, s>>>(L.cav, L.wave_cav, L.slow_list, L.n_slow);
        break;
    case KIND_AA_ODD:
        k_step_batch_slow<Q, MODEL, ST, KIND_AA_ODD><<<g, b, 0, s>>>(L.cav, L.wave_cav, L.slow_list, L.n_slow);
        break;
    case KIND_PULL:
        k_step_batch_slow<Q, MODEL, ST, KIND_PULL><<<g, b, 0, s>>>(L.cav, L.wave_cav, L.slow_list, L.n_slow);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q, class ST, int LAYOUT, int MODEL>
hipError_t launch_model(const Launch& L, hipStream_t s)
{
    const dim3 g(L.grid), b(L.block);
    switch (L.op) {
    case OP_STEP: return launch_step_kind<Q, MODEL, ST, LAYOUT>(L, s);
    case OP_STEP_SLOW: return launch_slow_kind<Q, MODEL, ST, LAYOUT>(L, s);
    case OP_STEP_ALL:
        if constexpr (Q == 19 && LAYOUT == LAYOUT_SOA) return launch_all_kind<Q, MODEL, ST, LAYOUT>(L, s);
        else return hipErrorInvalidValue;
    case OP_STEP_BATCH:
        if constexpr (Q == 19 && LAYOUT == LAYOUT_SOA) return launch_batch_kind<Q, MODEL, ST>(L, s);
        else return hipErrorInvalidValue;
    case OP_STEP_BATCH_SLOW:
        if constexpr (Q == 19 && LAYOUT == LAYOUT_SOA) return launch_batch_slow_kind<Q, MODEL, ST>(L, s);
        else return hipErrorInvalidValue;
    case OP_INIT: k_init<Q, MODEL, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.init); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

using LaunchFnPtr = hipError_t (*)(const Launch&, hipStream_t);

template <int Q, class ST, int LAYOUT>
hipError_t launch_layout(const Launch& L, hipStream_t s, LaunchFnPtr moment_space)
{
    const dim3 g(L.grid), b(L.block);
    switch (L.op) {
    case OP_GET: k_get_populations<Q, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.aa_odd, L.d0); break;
    case OP_MACRO: k_macroscopic<Q, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.aa_odd, L.d0, L.d1); break;
    case OP_SET: k_set_populations<Q, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.c0); break;
    case OP_INVARIANTS: k_invariants<Q, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.aa_odd, L.d0); break;
    case OP_NEIGHBORS: k_neighbors<Q><<<g, b, 0, s>>>(L.F, L.cells, L.n, L.idx_out); break;
    case OP_GET_CELLS: k_get_cells<Q, ST, LAYOUT><<<g, b, 0, s>>>(L.F, L.aa_odd, L.cells, L.n, L.d0); break;
    default:
        switch (L.model) {
        case BGK: return launch_model<Q, ST, LAYOUT, BGK>(L, s);
        case TRT: return launch_model<Q, ST, LAYOUT, TRT>(L, s);
        case REG: return launch_model<Q, ST, LAYOUT, REG>(L, s);
        case RR: return launch_model<Q, ST, LAYOUT, RR>(L, s);
        case NW4: case RM: case HM: case CM: case CHM: case CUM: return moment_space(L, s);
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// Model launches of the moment-space models, kept in translation units of
// their own (they are the largest kernels to compile).
template <int Q, class ST, int LAYOUT>
hipError_t launch_layout_moment_space(const Launch& L, hipStream_t s)
{
    switch (L.model) {
    case NW4: return launch_model<Q, ST, LAYOUT, NW4>(L, s);
    case RM: return launch_model<Q, ST, LAYOUT, RM>(L, s);
    case HM: return launch_model<Q, ST, LAYOUT, HM>(L, s);
    case CM: return launch_model<Q, ST, LAYOUT, CM>(L, s);
    case CHM: return launch_model<Q, ST, LAYOUT, CHM>(L, s);
    case CUM:
        if constexpr (Q == 19) return launch_model<Q, ST, LAYOUT, CUM>(L, s);
        else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <int Q, class ST>
hipError_t launch_tu(const Launch& L, hipStream_t s, LaunchFnPtr moment_space)
{
    if (L.layout == LAYOUT_SOA) return launch_layout<Q, ST, LAYOUT_SOA>(L, s, moment_space);
    if (L.layout == LAYOUT_AOS) return launch_layout<Q, ST, LAYOUT_AOS>(L, s, moment_space);
    if (L.layout == LAYOUT_BLOCKED) return launch_layout<Q, ST, LAYOUT_BLOCKED>(L, s, moment_space);
    return hipErrorInvalidValue;
}

template <int Q, class ST>
hipError_t launch_tu_moment_space(const Launch& L, hipStream_t s)
{
    if (L.layout == LAYOUT_SOA) return launch_layout_moment_space<Q, ST, LAYOUT_SOA>(L, s);
    if (L.layout == LAYOUT_AOS) return launch_layout_moment_space<Q, ST, LAYOUT_AOS>(L, s);
    if (L.layout == LAYOUT_BLOCKED) return launch_layout_moment_space<Q, ST, LAYOUT_BLOCKED>(L, s);
    return hipErrorInvalidValue;
}

}  // namespace lbm
