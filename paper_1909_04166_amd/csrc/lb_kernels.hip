// lb_kernels.hip -- instantiations and launchers of the step kernels (gfx950).
// The other kernels (state set-up and read-out, diagnostics, the built-in
// initial field, the copy reference) are in lb_aux.hip.
#include "lb_internal.hpp"

namespace cmlb {

// ------------------------------------------------------------ fused step

// The kernel behind a step: the coupled pair (lb_fused) or the phase field alone
// (lb_ace), with the cascaded or the SRT collisions.  The variant that prefetches
// rows (PF_PREFETCH) exists for the coupled cascaded kernel only.  W false: the
// launch's lattices have no walls (the kernels' wall logic is compiled out).  NT:
// nontemporal stores (coupled kernels whose strips are whole cache lines).
template <class ST, int TX, int MODE, int PF, int KIND, bool W, bool NT = false>
static void launch_one(dim3 grid, const LatDesc* d, const WorkItem* items, int n_items, int parity,
                       hipStream_t s) {
    if constexpr (KIND == KIND_COUPLED_CASCADED)
        hipLaunchKernelGGL((lb_fused<ST, TX, MODE, PF, COLL_CASCADED, W, NT>), grid, dim3(TX), 0, s, d, items, n_items,
                           parity);
    else if constexpr (KIND == KIND_COUPLED_SRT)
        hipLaunchKernelGGL((lb_fused<ST, TX, MODE, PF_HOLD, COLL_SRT, W, NT>), grid, dim3(TX), 0, s, d, items, n_items,
                           parity);
    else if constexpr (KIND == KIND_COUPLED_PRINTED)
        hipLaunchKernelGGL((lb_fused<ST, TX, MODE, PF_HOLD, COLL_PRINTED, W, NT>), grid, dim3(TX), 0, s, d, items,
                           n_items, parity);
    else if constexpr (KIND == KIND_ACE_CASCADED)
        hipLaunchKernelGGL((lb_ace<ST, TX, MODE, COLL_CASCADED, W>), grid, dim3(TX), 0, s, d, items, n_items, parity);
    else
        hipLaunchKernelGGL((lb_ace<ST, TX, MODE, COLL_SRT, W>), grid, dim3(TX), 0, s, d, items, n_items, parity);
}

// A width whose strips are whole cache lines, with or without nontemporal stores.
template <class ST, int TX, int MODE, int PF, int KIND, bool W>
static void launch_lines(bool nt, dim3 grid, const LatDesc* d, const WorkItem* items, int n_items, int parity,
                         hipStream_t s) {
    static_assert(kStripLines<ST, TX>, "strips of whole cache lines");
    if constexpr (MODE == MODE_STEP && KIND != KIND_ACE_CASCADED && KIND != KIND_ACE_SRT) {
        if (nt) {
            launch_one<ST, TX, MODE, PF, KIND, W, true>(grid, d, items, n_items, parity, s);
            return;
        }
    }
    launch_one<ST, TX, MODE, PF, KIND, W, false>(grid, d, items, n_items, parity, s);
}

template <class ST, int MODE, int PF, int KIND, bool W = true>
static hipError_t launch_tx(int tx, const LatDesc* d, const WorkItem* items, int n_items, int grid,
                            int parity, hipStream_t s, bool nt = false) {
    if (n_items <= 0) return hipSuccess;
    if (grid <= 0 || grid > n_items) grid = n_items;
    switch (tx) {
    case 64: launch_one<ST, 64, MODE, PF, KIND, W>(dim3(grid), d, items, n_items, parity, s); break;
    case 128: launch_one<ST, 128, MODE, PF, KIND, W>(dim3(grid), d, items, n_items, parity, s); break;
    case 256: launch_one<ST, 256, MODE, PF, KIND, W>(dim3(grid), d, items, n_items, parity, s); break;
    case 512: launch_one<ST, 512, MODE, PF, KIND, W>(dim3(grid), d, items, n_items, parity, s); break;
    // 64k + 4 lanes: strips of 64k columns, so every wave but the last works on
    // whole cache lines (see lane_slot); step kernels only
    case 132:
        if constexpr (MODE == MODE_STEP)
            launch_lines<ST, 132, MODE, PF, KIND, W>(nt, dim3(grid), d, items, n_items, parity, s);
        else
            return hipErrorInvalidValue;
        break;
    case 260:
        if constexpr (MODE == MODE_STEP)
            launch_lines<ST, 260, MODE, PF, KIND, W>(nt, dim3(grid), d, items, n_items, parity, s);
        else
            return hipErrorInvalidValue;
        break;
    case 452:
        if constexpr (MODE == MODE_STEP)
            launch_lines<ST, 452, MODE, PF, KIND, W>(nt, dim3(grid), d, items, n_items, parity, s);
        else
            return hipErrorInvalidValue;
        break;
    case 516:  // 9 waves: three per SIMD on one, at most 168 VGPRs (FP64 prefetching: 145)
        if constexpr (MODE == MODE_STEP)
            launch_lines<ST, 516, MODE, PF, KIND, W>(nt, dim3(grid), d, items, n_items, parity, s);
        else
            return hipErrorInvalidValue;
        break;
    case 1024:  // 16 waves: FP32 compute without prefetching only (4 waves per SIMD)
        if constexpr (sizeof(typename ST::R) == 4 && PF == PF_HOLD && MODE == MODE_STEP)
            launch_one<ST, 1024, MODE, PF, KIND, W>(dim3(grid), d, items, n_items, parity, s);
        else
            return hipErrorInvalidValue;
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class ST, bool W>
static hipError_t launch_step_kind(int kind, bool nt, int tx, int pf, const LatDesc* d, const WorkItem* items,
                                 int n_items, int grid, int parity, hipStream_t s) {
    switch (kind) {
    case KIND_COUPLED_CASCADED:
        if (pf == PF_PREFETCH)
            return launch_tx<ST, MODE_STEP, PF_PREFETCH, KIND_COUPLED_CASCADED, W>(tx, d, items, n_items, grid, parity, s,
                                                                                   nt);
        return launch_tx<ST, MODE_STEP, PF_HOLD, KIND_COUPLED_CASCADED, W>(tx, d, items, n_items, grid, parity, s, nt);
    case KIND_COUPLED_SRT:
        return launch_tx<ST, MODE_STEP, PF_HOLD, KIND_COUPLED_SRT, W>(tx, d, items, n_items, grid, parity, s, nt);
    case KIND_COUPLED_PRINTED:
        return launch_tx<ST, MODE_STEP, PF_HOLD, KIND_COUPLED_PRINTED, W>(tx, d, items, n_items, grid, parity, s, nt);
    case KIND_ACE_CASCADED:
        return launch_tx<ST, MODE_STEP, PF_HOLD, KIND_ACE_CASCADED, W>(tx, d, items, n_items, grid, parity, s);
    case KIND_ACE_SRT:
        return launch_tx<ST, MODE_STEP, PF_HOLD, KIND_ACE_SRT, W>(tx, d, items, n_items, grid, parity, s);
    }
    return hipErrorInvalidValue;
}

template <class ST>
static hipError_t launch_step_st(int kind, bool walls, bool nt, int tx, int pf, const LatDesc* d,
                                 const WorkItem* items, int n_items, int grid, int parity, hipStream_t s) {
    return walls ? launch_step_kind<ST, true>(kind, nt, tx, pf, d, items, n_items, grid, parity, s)
                 : launch_step_kind<ST, false>(kind, nt, tx, pf, d, items, n_items, grid, parity, s);
}

hipError_t launch_step(int prec, int kind, bool walls, bool nt, int tx, int pf, const LatDesc* d,
                       const WorkItem* items, int n_items, int grid, int parity, hipStream_t s) {
    switch (prec) {
    case LB_FP64: return launch_step_st<StF64>(kind, walls, nt, tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32: return launch_step_st<StF32>(kind, walls, nt, tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32_F16: return launch_step_st<StF16>(kind, walls, nt, tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32_BF16: return launch_step_st<StBF16>(kind, walls, nt, tx, pf, d, items, n_items, grid, parity, s);
    }
    return hipErrorInvalidValue;
}

template <class F>
static int occ_of(F kern, int tx) {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, tx, 0) == hipSuccess ? nb : 1;
}

template <class ST, int TX, bool W>
static int occ_kind(int kind, int pf) {
    switch (kind) {
    case KIND_COUPLED_CASCADED:
        if (pf == PF_PREFETCH) return occ_of(lb_fused<ST, TX, MODE_STEP, PF_PREFETCH, COLL_CASCADED, W>, TX);
        return occ_of(lb_fused<ST, TX, MODE_STEP, PF_HOLD, COLL_CASCADED, W>, TX);
    case KIND_COUPLED_SRT: return occ_of(lb_fused<ST, TX, MODE_STEP, PF_HOLD, COLL_SRT, W>, TX);
    case KIND_COUPLED_PRINTED: return occ_of(lb_fused<ST, TX, MODE_STEP, PF_HOLD, COLL_PRINTED, W>, TX);
    case KIND_ACE_CASCADED: return occ_of(lb_ace<ST, TX, MODE_STEP, COLL_CASCADED, W>, TX);
    case KIND_ACE_SRT: return occ_of(lb_ace<ST, TX, MODE_STEP, COLL_SRT, W>, TX);
    }
    return 1;
}

template <class ST, bool W>
static int occ_st(int kind, int tx, int pf) {
    switch (tx) {
    case 64: return occ_kind<ST, 64, W>(kind, pf);
    case 128: return occ_kind<ST, 128, W>(kind, pf);
    case 256: return occ_kind<ST, 256, W>(kind, pf);
    case 512: return occ_kind<ST, 512, W>(kind, pf);
    case 132: return occ_kind<ST, 132, W>(kind, pf);
    case 260: return occ_kind<ST, 260, W>(kind, pf);
    case 452: return occ_kind<ST, 452, W>(kind, pf);
    case 516: return occ_kind<ST, 516, W>(kind, pf);
    case 1024:
        if constexpr (sizeof(typename ST::R) == 4) {
            if (pf != PF_HOLD) return 0;
            switch (kind) {
            case KIND_COUPLED_CASCADED: return occ_of(lb_fused<ST, 1024, MODE_STEP, PF_HOLD, COLL_CASCADED, W>, 1024);
            case KIND_COUPLED_SRT: return occ_of(lb_fused<ST, 1024, MODE_STEP, PF_HOLD, COLL_SRT, W>, 1024);
            case KIND_COUPLED_PRINTED: return occ_of(lb_fused<ST, 1024, MODE_STEP, PF_HOLD, COLL_PRINTED, W>, 1024);
            case KIND_ACE_CASCADED: return occ_of(lb_ace<ST, 1024, MODE_STEP, COLL_CASCADED, W>, 1024);
            case KIND_ACE_SRT: return occ_of(lb_ace<ST, 1024, MODE_STEP, COLL_SRT, W>, 1024);
            }
        }
        return 0;
    }
    return 1;
}

template <bool W>
static int step_occupancy_w(int prec, int kind, int tx, int pf) {
    switch (prec) {
    case LB_FP64: return occ_st<StF64, W>(kind, tx, pf);
    case LB_FP32: return occ_st<StF32, W>(kind, tx, pf);
    case LB_FP32_F16: return occ_st<StF16, W>(kind, tx, pf);
    case LB_FP32_BF16: return occ_st<StBF16, W>(kind, tx, pf);
    }
    return 1;
}

int step_occupancy(int prec, int kind, bool walls, int tx, int pf) {
    return walls ? step_occupancy_w<true>(prec, kind, tx, pf) : step_occupancy_w<false>(prec, kind, tx, pf);
}

// Fields / coupling extraction always runs with 64-wide strips.  The coupled
// kinds share one extraction kernel (the fields do not depend on the collision).
template <class ST>
static hipError_t launch_extract_st(int kind, int mode, const LatDesc* d, const WorkItem* items64,
                                    int n_items, int parity, hipStream_t s) {
    const bool ace = kind == KIND_ACE_CASCADED || kind == KIND_ACE_SRT;
    if (mode == MODE_FIELDS)
        return ace ? launch_tx<ST, MODE_FIELDS, PF_HOLD, KIND_ACE_CASCADED>(64, d, items64, n_items, 0, parity, s)
                   : launch_tx<ST, MODE_FIELDS, PF_HOLD, KIND_COUPLED_CASCADED>(64, d, items64, n_items, 0, parity, s);
    return ace ? launch_tx<ST, MODE_COUPLING, PF_HOLD, KIND_ACE_CASCADED>(64, d, items64, n_items, 0, parity, s)
               : launch_tx<ST, MODE_COUPLING, PF_HOLD, KIND_COUPLED_CASCADED>(64, d, items64, n_items, 0, parity, s);
}

hipError_t launch_extract(int prec, int kind, int mode, const LatDesc* d, const WorkItem* items64,
                          int n_items, int parity, hipStream_t s) {
    switch (prec) {
    case LB_FP64: return launch_extract_st<StF64>(kind, mode, d, items64, n_items, parity, s);
    case LB_FP32: return launch_extract_st<StF32>(kind, mode, d, items64, n_items, parity, s);
    case LB_FP32_F16: return launch_extract_st<StF16>(kind, mode, d, items64, n_items, parity, s);
    case LB_FP32_BF16: return launch_extract_st<StBF16>(kind, mode, d, items64, n_items, parity, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cmlb
