// Kernel launchers of the single-instance path: the launch shape of the
// iteration, check and plan kernels, the template ladders that map a shape
// onto a kernel instantiation, and the cooperative kernel of a cost source.
// Their kernel instantiations are compiled in launch_dense.hip,
// launch_rates.hip and launch_geo.hip (one cost source family each, built in
// parallel); ot_assoc.hip declares them with OT_LAUNCHERS(extern, ...).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "handle.h"
#include "kernels.h"
#include "persist_kernels.h"

namespace otk_launch {
using namespace otk;

constexpr int kMaxNb = 1024;  // workgroups per sweep (partial rows)
constexpr int kPersistWaves = 8;

inline int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// ------------------------------------------------------------- launch shape --
struct Shape {
    int vec = 1, lpr = 64, nch = 1, nchT = 1, waves = 8, nb = 1, rb = 1;
    int64_t rpb = 1;
};

// Vector width of the row loads: 16-byte loads need J and the row stride to
// be multiples of the width and an aligned base, so that no vector straddles
// J (padding entries are never read as costs).
template <class Src>
int vec_for(int64_t J, int64_t ld, const void* d) {
    if (Src::kVecWide == 1) return 1;
    const int w = Src::kVecWide;
    return (J % w == 0 && ld % w == 0 && ((uintptr_t)d % 16) == 0) ? w : 1;
}

inline int64_t ld_of(const ot_cost_desc& c) { return c.ld ? c.ld : c.J; }

template <class Src>
constexpr int max_rb(bool p64) {
    return Src::kCheap ? (p64 ? 2 : (Src::kTag == 1 || Src::kTag == 3 ? 8 : 2)) : 1;
}
constexpr int max_nch(int vec, int lpr) { return lpr < 64 ? 8 : 2048 / (64 * vec); }

// Iteration shape: a row per group of LPR lanes (the narrowest of 16 and 32
// that keeps at most 4 column chunks of LPR * VEC, else at most 8, else 64
// lanes), contiguous row ranges per workgroup, RB steps of rows in flight per
// wave. The grid is sized afterwards by fit_grid.
template <class Src>
Shape make_shape(const ot_assoc* h, int64_t I, int64_t J, int vec, bool p64 = false) {
    Shape s;
    s.vec = vec;
    s.lpr = 64;
    for (int lim : {4, 8}) {  // prefer at most 4 column chunks per lane (register budget)
        for (int cand : {16, 32})
            if ((J + cand * vec - 1) / (cand * vec) <= lim) { s.lpr = cand; break; }
        if (s.lpr < 64) break;
    }
    if (h->opt.sweep_lanes == 16 || h->opt.sweep_lanes == 32 || h->opt.sweep_lanes == 64)
        if ((J + h->opt.sweep_lanes * vec - 1) / (h->opt.sweep_lanes * vec) <= max_nch(vec, h->opt.sweep_lanes))
            s.lpr = h->opt.sweep_lanes;
    s.nch = (int)((J + s.lpr * vec - 1) / (s.lpr * vec));
    s.nchT = pow2_at_least(s.nch);
    if (s.lpr == 64) s.nchT = std::max(s.nchT, vec == 1 ? 4 : 8);  // the instantiated widths
    s.waves = (Src::kTag == 1 && h->opt.sweep_waves > 0) ? h->opt.sweep_waves : 8;
    const int R = 64 / s.lpr;
    int nb = h->opt.sweep_blocks > 0 ? h->opt.sweep_blocks : 512;
    nb = (int)std::min<int64_t>(nb, (I + s.waves * R - 1) / (s.waves * R));
    nb = std::max(1, std::min(nb, kMaxNb));
    s.rpb = (I + nb - 1) / nb;
    s.nb = (int)((I + s.rpb - 1) / s.rpb);
    const int steps = (int)((s.rpb + s.waves * R - 1) / (s.waves * R));
    // one step in flight measured best whenever a row is shared by lanes (the
    // registers of a second step cost more occupancy than they hide latency)
    const int want = h->opt.sweep_rows > 0 ? h->opt.sweep_rows : (s.lpr < 64 ? 1 : pow2_at_least(steps));
    const int cap = (s.lpr < 64) ? 2 : std::max(1, 16 / s.nchT);
    s.rb = std::min({want, max_rb<Src>(p64), cap});
    return s;
}

// LDS of the iteration kernel: staged per-column source data and g in FP64
// and FP32, reused afterwards by the workgroup reduction tree.
template <class Src>
size_t sweep_lds(const Shape& s, bool p64) {
    const size_t ncols = (size_t)s.nch * s.lpr * s.vec;
    const size_t a = sizeof(double) * ((size_t)Src::kStageDoubles * ncols + ncols + (ncols + 1) / 2);
    const size_t b = (p64 ? sizeof(double) : sizeof(float)) * (size_t)s.waves * (64 / s.lpr) * ncols;
    return std::max(a, b);
}

// The check and plan kernels use one 64-lane wavefront per row.
inline Shape row64(Shape s, int64_t J) {
    s.lpr = 64;
    s.nch = (int)((J + 64 * s.vec - 1) / (64 * s.vec));
    s.nchT = pow2_at_least(s.nch);
    return s;
}

// LDS of the check kernel (64 lanes per row): staged data plus the reduction tree.
template <class Src>
size_t check_lds(const Shape& s) {
    const size_t ncols = (size_t)s.nch * 64 * s.vec;
    return sizeof(double) * std::max((size_t)(Src::kStageDoubles + 1) * ncols, (size_t)4 * ncols);
}

// While set, the launch helpers only raise the kernels' LDS limits and launch
// nothing: run before a graph capture so no attribute call happens inside it.
inline thread_local bool g_prepare_only = false;

template <class K>
void set_lds(K kern, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// While set, the iteration launcher stores the kernel's resident workgroups
// per CU here instead of launching (used to size the grid to one full wave).
inline thread_local int* g_occupancy_query = nullptr;

template <class Src, bool P64, int VEC, int NCH, int LPR, int W, int RB>
void launch_iter_t(const Shape& s, const IterArgs& A, const Src& src, size_t lds, hipStream_t st) {
    auto kern = k_iter<Src, P64, VEC, NCH, LPR, W, RB>;
    set_lds(kern, lds);
    if (g_occupancy_query) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, W * 64, lds) != hipSuccess) n = 0;
        *g_occupancy_query = n;
        return;
    }
    if (g_prepare_only) return;
    hipLaunchKernelGGL(kern, dim3(s.nb), dim3(W * 64), lds, st, A, src);
}

template <class Src, bool P64, int VEC, int NCH, int LPR, int W>
bool launch_iter_r(const Shape& s, const IterArgs& A, const Src& src, size_t lds, hipStream_t st) {
    constexpr int kMaxRb = std::min(max_rb<Src>(P64), LPR < 64 ? 2 : std::max(1, 16 / NCH));
    switch (s.rb) {
        case 1: launch_iter_t<Src, P64, VEC, NCH, LPR, W, 1>(s, A, src, lds, st); return true;
        case 2: if constexpr (kMaxRb >= 2) { launch_iter_t<Src, P64, VEC, NCH, LPR, W, 2>(s, A, src, lds, st); return true; } break;
        case 4: if constexpr (kMaxRb >= 4) { launch_iter_t<Src, P64, VEC, NCH, LPR, W, 4>(s, A, src, lds, st); return true; } break;
        case 8: if constexpr (kMaxRb >= 8) { launch_iter_t<Src, P64, VEC, NCH, LPR, W, 8>(s, A, src, lds, st); return true; } break;
    }
    return false;
}

template <class Src, bool P64, int VEC, int LPR, int W>
bool launch_iter_n(const Shape& s, const IterArgs& A, const Src& src, size_t lds, hipStream_t st) {
    if constexpr (LPR < 64) {
        switch (s.nchT) {
            case 1: return launch_iter_r<Src, P64, VEC, 1, LPR, W>(s, A, src, lds, st);
            case 2: return launch_iter_r<Src, P64, VEC, 2, LPR, W>(s, A, src, lds, st);
            case 4: return launch_iter_r<Src, P64, VEC, 4, LPR, W>(s, A, src, lds, st);
            case 8: return launch_iter_r<Src, P64, VEC, 8, LPR, W>(s, A, src, lds, st);
        }
    } else {
        switch (s.nchT) {
            case 4: if constexpr (VEC == 1) return launch_iter_r<Src, P64, VEC, 4, LPR, W>(s, A, src, lds, st); break;
            case 8: return launch_iter_r<Src, P64, VEC, 8, LPR, W>(s, A, src, lds, st);
            case 16: if constexpr (VEC <= 2) return launch_iter_r<Src, P64, VEC, 16, LPR, W>(s, A, src, lds, st); break;
            case 32: if constexpr (VEC == 1) return launch_iter_r<Src, P64, VEC, 32, LPR, W>(s, A, src, lds, st); break;
        }
    }
    return false;
}

template <class Src, bool P64, int VEC, int W>
bool launch_iter_l(const Shape& s, const IterArgs& A, const Src& src, size_t lds, hipStream_t st) {
    switch (s.lpr) {
        case 16: return launch_iter_n<Src, P64, VEC, 16, W>(s, A, src, lds, st);
        case 32: return launch_iter_n<Src, P64, VEC, 32, W>(s, A, src, lds, st);
        case 64: return launch_iter_n<Src, P64, VEC, 64, W>(s, A, src, lds, st);
    }
    return false;
}

template <class Src, bool P64, int VEC>
bool launch_iter_v(const Shape& s, const IterArgs& A, const Src& src, size_t lds, hipStream_t st) {
    if constexpr (Src::kTag == 1) {  // the dense FP32 hot path is tunable in waves per workgroup
        if (s.waves == 4) return launch_iter_l<Src, P64, VEC, 4>(s, A, src, lds, st);
    }
    if (s.waves == 8) return launch_iter_l<Src, P64, VEC, 8>(s, A, src, lds, st);
    return false;
}

template <class Src, bool P64>
bool launch_iter(const Shape& s, const IterArgs& A, const Src& src, hipStream_t st) {
    const size_t lds = sweep_lds<Src>(s, P64);
    if (s.vec == 1) return launch_iter_v<Src, P64, 1>(s, A, src, lds, st);
    if constexpr (Src::kVecWide > 1)
        if (s.vec == Src::kVecWide) return launch_iter_v<Src, P64, Src::kVecWide>(s, A, src, lds, st);
    return false;
}

template <int VEC>
constexpr int check_nch() { return VEC == 4 ? 8 : VEC == 2 ? 16 : 32; }  // J <= 2048

// Whether the check of this shape can also sum the RRH loads: only the
// narrow instantiation (J <= 512) has the registers for a second set of
// column accumulators; the wide one is at the register limit without them
// (with them it spills, at eight waves and at four).
inline bool check_fuses_loads(const Shape& s) {
    const int wide = s.vec == 4 ? 8 : s.vec == 2 ? 16 : 32;
    return s.lpr == 64 && s.nch <= wide / 4;
}

template <class Src, int VEC>
bool launch_check_v(const Shape& s, const CheckArgs& A, const Src& src, hipStream_t st) {
    const size_t lds = check_lds<Src>(s);
    // narrow instances (up to a quarter of the column capacity, e.g. J <= 512
    // at VEC 4) take an instantiation with a quarter of the per-lane column
    // registers: at 20000 x 400 the wide one holds 241 VGPRs (2 waves / SIMD)
    constexpr int kWide = check_nch<VEC>(), kNarrow = kWide / 4;
    if (A.load_part) {  // the check that also sums the RRH loads (narrow instances only)
        if (s.nch > kNarrow) return false;
        auto kern = k_check<Src, VEC, kNarrow, 8, true>;
        set_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3(s.nb), dim3(512), lds, st, A, src);
        return true;
    }
    if (A.plan_out) {  // the check that also writes the plan
        auto pick = [&](auto narrow, auto wide) {
            auto kern = s.nch <= kNarrow ? narrow : wide;
            set_lds(kern, lds);
            hipLaunchKernelGGL(kern, dim3(s.nb), dim3(512), lds, st, A, src);
        };
        if (A.plan_f64) pick(k_check<Src, VEC, kNarrow, 8, false, double>, k_check<Src, VEC, kWide, 8, false, double>);
        else pick(k_check<Src, VEC, kNarrow, 8, false, float>, k_check<Src, VEC, kWide, 8, false, float>);
        return true;
    }
    if (s.nch <= kNarrow) {
        auto kern = k_check<Src, VEC, kNarrow, 8>;
        set_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3(s.nb), dim3(512), lds, st, A, src);
        return true;
    }
    auto kern = k_check<Src, VEC, kWide, 8>;
    set_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3(s.nb), dim3(512), lds, st, A, src);
    return true;
}

template <class Src>
bool launch_check(const Shape& s, const CheckArgs& A, const Src& src, hipStream_t st) {
    if (s.vec == 1) return launch_check_v<Src, 1>(s, A, src, st);
    if constexpr (Src::kVecWide > 1)
        if (s.vec == Src::kVecWide) return launch_check_v<Src, Src::kVecWide>(s, A, src, st);
    return false;
}

// Plan rows [r0, r1) into `out` (row r0 first).
template <class Src, typename OutT, int VEC>
void launch_plan_v(const Shape& s, int64_t r0, int64_t r1, int J, const double* f, const double* g,
                   const SolveParams* prm, OutT* out, const Src& src, hipStream_t st) {
    const size_t ncols = (size_t)s.nch * 64 * VEC;
    const size_t lds = sizeof(double) * (Src::kStageDoubles + 1) * ncols;
    auto kern = k_plan<Src, OutT, VEC>;
    set_lds(kern, lds);
    const int grid = (int)std::min<int64_t>(4096, (r1 - r0 + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(512), lds, st, r0, r1, J, s.nch, f, g, prm, out, src);
}

template <class Src, typename OutT>
bool launch_plan(const Shape& s, int64_t r0, int64_t r1, int J, const double* f, const double* g,
                 const SolveParams* prm, OutT* out, const Src& src, hipStream_t st) {
    if (s.vec == 1) { launch_plan_v<Src, OutT, 1>(s, r0, r1, J, f, g, prm, out, src, st); return true; }
    if constexpr (Src::kVecWide > 1)
        if (s.vec == Src::kVecWide) {
            launch_plan_v<Src, OutT, Src::kVecWide>(s, r0, r1, J, f, g, prm, out, src, st);
            return true;
        }
    return false;
}


// Shape of the LDS-resident FP32 phase: one workgroup of kPersistWaves waves
// per CU, rows per workgroup a whole number of wave steps; lanes per row and
// cells per lane by J (column q LPR + sub of a row belongs to lane sub).
// Sources whose fast-sweep cost is an FP32 value (dense FP32, FP32 rates, the
// FP32 geometry and distance functors): the tile holds exactly what the
// streaming sweeps compute per cell.
template <class Src>
constexpr bool persist_source() { return Src::kTag == 1 || Src::kTag == 3 || Src::kTag == 5 || Src::kTag == 6; }

template <class Src>
const void* persist_kernel(int lpr, int cpl) {
    if constexpr (!persist_source<Src>()) {
        return nullptr;
    } else {
    if (lpr == 32) {
        switch (cpl) {
            case 2: return (const void*)k_persist<Src, 2, 32, kPersistWaves>;
            case 4: return (const void*)k_persist<Src, 4, 32, kPersistWaves>;
            case 8: return (const void*)k_persist<Src, 8, 32, kPersistWaves>;
            case 13: return (const void*)k_persist<Src, 13, 32, kPersistWaves>;
            default: return (const void*)k_persist<Src, 16, 32, kPersistWaves>;
        }
    }
    if (cpl == 16) return (const void*)k_persist<Src, 16, 64, kPersistWaves>;
    return (const void*)k_persist<Src, 32, 64, kPersistWaves>;
    }
}

}  // namespace otk_launch

// Explicit instantiation (EXT empty) or its declaration (EXT = extern) of
// every launcher of cost source S.
#define OT_LAUNCHERS(EXT, S)                                                                                       \
    EXT template bool otk_launch::launch_iter<S, false>(const otk_launch::Shape&, const otk::IterArgs&, const S&,  \
                                                        hipStream_t);                                              \
    EXT template bool otk_launch::launch_iter<S, true>(const otk_launch::Shape&, const otk::IterArgs&, const S&,   \
                                                       hipStream_t);                                               \
    EXT template bool otk_launch::launch_check<S>(const otk_launch::Shape&, const otk::CheckArgs&, const S&,       \
                                                  hipStream_t);                                                    \
    EXT template bool otk_launch::launch_plan<S, float>(const otk_launch::Shape&, int64_t, int64_t, int,            \
                                                        const double*, const double*, const otk::SolveParams*,     \
                                                        float*, const S&, hipStream_t);                            \
    EXT template bool otk_launch::launch_plan<S, double>(const otk_launch::Shape&, int64_t, int64_t, int,           \
                                                         const double*, const double*, const otk::SolveParams*,    \
                                                         double*, const S&, hipStream_t);                          \
    EXT template const void* otk_launch::persist_kernel<S>(int, int);
