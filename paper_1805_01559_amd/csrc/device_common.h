// Device-side helpers shared by the association kernels: wavefront (64-lane)
// reductions, the per-solve control block and the constants of the log2
// domain in which every exponential is taken.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace otk {

constexpr int kWave = 64;
constexpr double kLog2e = 1.4426950408889634074;  // 1 / ln 2
constexpr double kLn2 = 0.69314718055994530942;

// 2^t in FP64 by table-driven reduction (P. T. P. Tang, "Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic", ACM TOMS 15(2), 1989): t = n + j / 64 + r with |r| <= 1/128,
// 2^(j/64) from a table of 64 entries (tab, filled by exp2_tab_fill), and
// 2^r - 1 from the Taylor polynomial of degree 6 in x = r ln 2 (|x| < 0.0055,
// truncation below 3e-20 relative). About 1 ulp; about half the FP64
// instructions of the library's exp2. For finite t only (results below the
// smallest subnormal round through ldexp to 0, above the largest double to
// infinity); callers select away lanes whose t is not finite.
__device__ __forceinline__ double exp2_tab(double t, const double* tab) {
    const double k = __builtin_rint(t * 64.0);
    const double r = fma(k, -1.0 / 64.0, t);  // exact for |t| < 2^46
    // (the conversion is clamped to keep it defined: beyond |t| = 2^14 the
    // result is 0 or infinity either way, and a NaN t stays NaN through q)
    const int ki = (int)fmin(fmax(k, -1048576.0), 1048576.0);
    const int j = ki & 63, n = ki >> 6;
    const double x = r * kLn2;
    double q = fma(x, 1.0 / 720.0, 1.0 / 120.0);
    q = fma(x, q, 1.0 / 24.0);
    q = fma(x, q, 1.0 / 6.0);
    q = fma(x, q, 0.5);
    q = fma(x, q, 1.0);
    q *= x;
    const double T = tab[j];
    return ldexp(fma(T, q, T), n);
}
// Fills tab[j] = 2^(j/64), j < 64, by the first 64 threads of the workgroup;
// the caller synchronises before use.
__device__ __forceinline__ void exp2_tab_fill(double* tab) {
    if (threadIdx.x < 64) tab[threadIdx.x] = exp2((double)threadIdx.x / 64.0);
}

// ---------------------------------------------------------------- reductions
// Reductions over the 64 lanes of a wavefront with DPP lane moves: xor-1 and
// xor-2 quad permutes, the 8-lane half-row mirror and the 16-lane row mirror
// leave every row of 16 lanes holding its row total; the four row totals are
// then read out and combined as (r0 + r1) + (r2 + r3). Every lane ends with
// the same value, in the same order on every call, so results are bitwise
// reproducible. DPP control codes: quad_perm(1,0,3,2) = 0xB1,
// quad_perm(2,3,0,1) = 0x4E, row_mirror = 0x140, row_half_mirror = 0x141.
// Each of these reads a lane of the same 16-lane row, and every row and bank
// is enabled, so no lane keeps its old value: the moves need no old operand.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    static_assert(CTRL == 0xB1 || CTRL == 0x4E || CTRL == 0x140 || CTRL == 0x141, "in-row DPP moves only");
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    static_assert(CTRL == 0xB1 || CTRL == 0x4E || CTRL == 0x140 || CTRL == 0x141 || CTRL == 0x128,
                  "in-row DPP moves only");
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_f(float x, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); }

// Pair sums across lanes with gfx950's row swaps (v_permlane16_swap,
// v_permlane32_swap: VALU moves) instead of LDS permutes. xor16_sum gives
// every lane v[l] + v[l ^ 16] and xor32_sum v[l] + v[l ^ 32], with the lower
// lane's value first in both lanes of a pair (so both hold the same bits).
__device__ __forceinline__ double xor16_sum(double v) {
    const long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);  // lower lane's value
    const double y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);  // upper lane's value
    return x + y;
}
__device__ __forceinline__ double xor32_sum(double v) {
    const long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
    const double y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
    return x + y;
}
__device__ __forceinline__ float xor32_sum(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));
    v = fmaxf(v, dpp_f<0x4E>(v));
    v = fmaxf(v, dpp_f<0x141>(v));
    v = fmaxf(v, dpp_f<0x140>(v));
    return fmaxf(fmaxf(readlane_f(v, 0), readlane_f(v, 16)), fmaxf(readlane_f(v, 32), readlane_f(v, 48)));
}

// Reductions over a group of LPR (16, 32 or 64) consecutive lanes; every lane
// of the group ends with the group's value. Within 16 lanes the same DPP
// steps as above; wider groups add xor-16 and xor-32 exchanges. Each step
// combines a lane's value with its partner's, so all lanes of a group agree.
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    if constexpr (LPR >= 32) v = xor16_sum(v);
    if constexpr (LPR >= 64) v = xor32_sum(v);
    return v;
}
template <int LPR>
__device__ __forceinline__ float group_max(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));
    v = fmaxf(v, dpp_f<0x4E>(v));
    v = fmaxf(v, dpp_f<0x141>(v));
    v = fmaxf(v, dpp_f<0x140>(v));
    if constexpr (LPR >= 32) v = fmaxf(v, __shfl_xor(v, 16, 64));
    if constexpr (LPR >= 64) v = fmaxf(v, __shfl_xor(v, 32, 64));
    return v;
}
template <int LPR>
__device__ __forceinline__ double group_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    if constexpr (LPR >= 32) v = fmax(v, __shfl_xor(v, 16, 64));
    if constexpr (LPR >= 64) v = fmax(v, __shfl_xor(v, 32, 64));
    return v;
}

// 2^x for x <= 0 in FP32 (one v_exp_f32).
__device__ __forceinline__ float exp2_f32(float x) { return __builtin_amdgcn_exp2f(x); }

// Per-solve constants read by the kernels.
struct SolveParams {
    double kk;   // log2(e) / eps
    double eps;
};

// ------------------------------------------------------------- control block
// Per-solve state that lives in device memory so that a captured chunk of
// iterations can decide on the device when to stop, without a host round
// trip per iteration.
enum : int {
    kModeFast = 0,    // FP32 sweeps: stop the chunk when the residual meets tol or stalls
    kModePolish = 1,  // FP64 sweeps run unconditionally (no stop decision)
    kModeExact = 2,   // FP64 sweeps: stop when an FP64 iterate meets tol
};

struct Ctl {
    int32_t iter;          // full iterations completed (the current iterate's number)
    int32_t stop;          // 1: remaining launches of the current chunk do nothing
    int32_t done;          // 1: converged (or failed); result_iter names the iterate
    int32_t result_iter;   // iterate to return when done
    int32_t numeric_bad;   // a non-finite value appeared
    int32_t fp64_iters;    // FP64 sweeps completed
    int32_t last_fp64;     // 1 if the current iterate came from an FP64 sweep
    int32_t max_iter;
    uint32_t arrive;       // last-block-done counter of the combine kernel
    uint32_t arrive2;      // same, for the check kernel
    int32_t has_prev;      // 1 if a previous iterate f^(k-1) exists (k >= 1 or warm start)
    int32_t check_every;   // the stop rule is evaluated after iterations k with k % check_every == 0 (0, 1: every k)
    double tol;
    double mass;           // sum(a)
    double r_last;         // residual of iterate (iter - 1), measured during iteration iter
    double r_hist[4];      // recent fast-mode residuals (stall detection)
    // results of the exact check of the current iterate
    double chk_violation, chk_objective, chk_reg_objective, chk_dual, chk_mass;
    double chk_row_res, chk_col_res;
    // per-instance phase of the batched engine (unused by single solves)
    int32_t phase;         // kPhFast .. kPhDone
    int32_t polish_left;   // FP64 polish sweeps still to run
    int32_t check_iter;    // iterate the pending check examines
    int32_t exact_done;    // 1: the next check ends the solve whatever it finds
    // single solves: inputs rejected on the device (bits: 1 a, 2 b, 4 sum a != sum b,
    // 8 cost or positions), and a cooperative launch whose grid barrier gave up
    int32_t input_bad;
    int32_t sync_fail;
    double mass_b;         // sum(b)
    // target of the FP32 phase. Single solves: tol / 4 when that is above
    // the FP32 noise threshold (the exact check that follows measures the row
    // AND column residual of the next iterate; a margin lets it pass the first
    // time instead of sending the solve into an FP64 phase with host round
    // trips), else tol. Batched instances: tol.
    double tol_fast;
};

// The FP32 phase's residual target for a solve to `tol`.
__host__ __device__ inline double fast_target(double tol, double stall_below) {
    return tol * 0.25 >= stall_below ? tol * 0.25 : tol;
}

}  // namespace otk
