// Association kernels for gfx950: one launch per Sinkhorn iteration (fused
// row update, column partials and the column combine), the exact FP64 check
// of an iterate, the plan writer and the per-instance set-up passes.
//
// Iteration k of the Sinkhorn algorithm (Sec. III-B), in log-domain form with
// FP64 potentials (f = eps log of the row scaling, g = eps log of the column
// scaling), is two launches:
//
//  k_iter    one read (or regeneration) of C per iteration. For every row i,
//            in base 2 with kk = log2(e) / eps,
//              t_ij = g_j kk - C_ij kk,  m_i = max_j t_ij,
//              e_ij = 2^(t_ij - m_i),   s_i = sum_j e_ij,
//              f_i  = eps (ln a_i - ln 2 (m_i + log2 s_i))      (row update)
//            and, from the same registers, the half-iterate plan entries
//              pi_ij = exp((f_i + g_j - C_ij)/eps) = e_ij a_i / s_i,
//            summed per column over the workgroup's rows. The row residual
//            |rowsum_i(pi^(k-1)) - a_i| = a_i |expm1((f_i^(k-1) - f_i)/eps)| of the
//            previous full iterate falls out of the change in f.
//  k_colsum  a second, small launch: each workgroup owns a slice of columns and
//            sums all workgroup partials of them in a fixed order, then
//              g_j <- g_j + eps (ln b_j - ln colsum_j)               (column update)
//            which is exactly eps ln b_j - eps LSE_i((f_i - C_ij)/eps). Its
//            first workgroup also sums the row residuals and takes the stop
//            decision for the chunk of iterations in flight.
//
// The exponentials e_ij are FP32 (v_exp_f32) in the fast sweeps and FP64 in
// the polish sweeps; arguments t_ij and every accumulation across lanes,
// rows and workgroups are FP64. Every reduction has a fixed order, so results
// are bitwise reproducible for a given launch shape. Workgroups never exchange
// data inside a launch: on this GPU a device-scope fence writes back the
// whole L2 of its XCD, so cross-workgroup results travel through the kernel
// boundary instead.
#pragma once

#include <type_traits>

#include "cost_sources.h"
#include "device_common.h"

namespace otk {

// ------------------------------------------------- block-level reductions --
// Sums acc[NCH][VEC] over the WAVES waves of a workgroup through LDS in a
// fixed tree order; wave 0 ends with the block total.
template <int NCH, int VEC, int WAVES>
__device__ __forceinline__ void block_tree(double (&acc)[NCH][VEC], int nch, double* red, int ncols, int w, int lane) {
#pragma unroll
    for (int half = WAVES / 2; half >= 1; half >>= 1) {
        if (w >= half && w < 2 * half) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) red[(w - half) * ncols + (ch * kWave + lane) * VEC + v] = acc[ch][v];
        }
        __syncthreads();
        if (w < half) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[ch][v] += red[w * ncols + (ch * kWave + lane) * VEC + v];
        }
        __syncthreads();
    }
}

// Fixed-order sum of rows [q0, q1) of a row-major (rows x J) array, column j.
__device__ __forceinline__ double sum_rows(const double* p, int q0, int q1, int J, int j) {
    double s = 0.0;
    int q = q0;
    for (; q + 8 <= q1; q += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = p[(int64_t)(q + u) * J + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; q < q1; ++q) s += p[(int64_t)q * J + j];
    return s;
}

// ------------------------------------------------------------ iteration --
struct IterArgs {
    int64_t I;
    int J;
    int nch;  // column chunks of 64 * VEC actually used (<= NCH)
    int64_t rows_per_block;
    const double* a;
    const double* la;    // ln a_i (or null)
    const double* f_in;  // f^(k-1) (read only when ctl->has_prev)
    double* f_out;       // f^k
    const double* g_in;  // g^(k-1)
    double* col_part;    // gridDim.x x J partial column sums of the half-iterate
    double* res_part;    // gridDim.x partial row residuals of iterate k-1
    const Ctl* ctl;
    const SolveParams* prm;
};

__device__ __forceinline__ void bookkeep(Ctl* c, double rsum, int mode, double stall_below) {
    const int k = c->iter + 1;
    const double r = c->has_prev ? rsum / c->mass : pinf64();
    const bool bad = c->numeric_bad || (c->has_prev && !isfinite(r));
    const int prev64 = c->last_fp64;
    c->r_last = r;
    c->iter = k;
    c->has_prev = 1;
    if (mode == kModeFast) {
        c->last_fp64 = 0;
        // stalled: the residual sits below the FP32 noise threshold and no
        // longer falls against the recent (finite) residuals
        double mn = pinf64();
        int nfin = 0;
        for (int q = 0; q < 4; ++q)
            if (isfinite(c->r_hist[q])) { mn = fmin(mn, c->r_hist[q]); ++nfin; }
        const bool stall = (nfin >= 1) && isfinite(r) && (r < stall_below) && (r > 0.95 * mn);
        for (int q = 3; q > 0; --q) c->r_hist[q] = c->r_hist[q - 1];
        c->r_hist[0] = r;
        const double target = c->tol_fast > 0.0 ? c->tol_fast : c->tol;
        const bool at_check = c->check_every <= 1 || k % c->check_every == 0;
        if ((at_check && (r < target || stall)) || k >= c->max_iter) c->stop = 1;
    } else {
        c->fp64_iters += 1;
        c->last_fp64 = 1;
        // (r is the residual of iterate k - 1, the one an exact stop returns)
        const bool at_check = c->check_every <= 1 || (k - 1) % c->check_every == 0;
        if (mode == kModeExact && prev64 && r < c->tol && at_check) {
            c->done = 1;
            c->stop = 1;
            c->result_iter = k - 1;
        } else if (k >= c->max_iter) {
            c->stop = 1;
        }
    }
    if (bad) {
        c->numeric_bad = 1;
        c->done = 1;
        c->stop = 1;
        c->result_iter = k;
    }
}

// Lane layout: a row is handled by a group of LPR lanes (16, 32 or 64), so a
// wavefront advances R = 64 / LPR rows per step; lane `sub` of a group owns
// columns (ch * LPR + sub) * VEC + v. Short rows (a few hundred RRHs) thus
// share one instruction stream four or two at a time, which amortises the
// per-row reductions and scalars over more cells. Each wave keeps RB steps of
// rows in flight and refills a slot as soon as its row is consumed.
// One workgroup's share of a sweep: rows [r0, r1) of one instance, with the
// column partials and the residual partial of those rows as outputs.
struct SweepJob {
    int64_t r0, r1;
    int J;
    int nch;
    int has_prev;               // used when prev_ctl is null
    const Ctl* prev_ctl;        // else has_prev is read from here
    const SolveParams* prm;     // kk, eps (read after the first loads are issued)
    const double* a;
    const double* la;           // ln a_i, or null: the FP32 sweeps then shift every row by its maximum
    const double* f_in;
    double* f_out;
    const double* g_in;
    double* col_part;  // rows of J partial column sums of the half-iterate ...
    double* res_part;  // ... and partial row residuals of the previous iterate
    int part;          // the row of both that this job writes
};

// The sweep of rows [r0, r1) by one workgroup. With stop_ctl set, the first
// loads are issued before the control block is read and the workgroup does
// nothing more if the chunk has been stopped. LDS is reused from the previous
// call of a persistent workgroup only after a barrier.
template <class Src, bool P64, int VEC, int NCH, int LPR, int WAVES, int RB, bool LSE>
__device__ __forceinline__ void sweep_rows(const SweepJob& A, const Src& src, const Ctl* stop_ctl) {
    // (the dynamic LDS is named here rather than passed in: a pointer
    // parameter loses its address space and turns LDS accesses into flat ones)
    extern __shared__ double sm[];
    constexpr int R = kWave / LPR;
    const int J = A.J, nch = A.nch;
    const int ncols = nch * LPR * VEC;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int sub = lane % LPR, rg = lane / LPR;
    const int64_t r0 = A.r0, r1 = A.r1;
    // first row of step `st` for this wave; this lane's row is that + rg
    auto step_base = [&](int64_t st) { return r0 + (st * WAVES + w) * R; };

    // 1. issue the loads of this wave's first RB steps before anything else;
    //    a slot holds a step's row data and its a_i (rows past the range load
    //    as fully masked, i.e. C = +inf, and get a_i = 0)
    using Raw = typename Src::template Raw<VEC>;
    Raw raw[RB][NCH];
    double aq[RB], lq[RB], fq[RB];
    // With LSE (FP32 sweeps) and ln a known, a row is shifted by its
    // log-sum-exp of the previous sweep, recovered from f: log2 sum_j
    // 2^(g_j kk - C_ij kk) = log2(e) ln a_i - kk f_i. That replaces the pass
    // over the row for its maximum, which runs only without a previous
    // iterate or when a row sum leaves [2^-100, 2^100] (the wave's rows are
    // then redone). (It pays where the sweep is bound by instruction issue;
    // sources that compute their costs and the batch kernel, whose registers
    // are already at their occupancy limit, keep the maximum.)
    static_assert(!(LSE && P64), "the log-sum-exp shift is for FP32 sweeps");
    const bool lse_ok = LSE && A.la != nullptr;
    auto issue = [&](int q, int64_t i) {
        const bool ok = i < r1;
        const int64_t ii = ok ? i : r0;
        auto row = src.row(ii);
        const int Jl = ok ? J : 0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (ch < nch) raw[q][ch] = src.template load<VEC>(row, (ch * LPR + sub) * VEC, Jl);
        aq[q] = ok ? A.a[i] : 0.0;
        if (lse_ok) {
            lq[q] = A.la[ii];
            fq[q] = A.f_in[ii];
        }
    };
#pragma unroll
    for (int q = 0; q < RB; ++q) issue(q, step_base(q) + rg);
    // a stopped chunk does nothing (the loads above are simply dropped)
    if (stop_ctl && (stop_ctl->stop | stop_ctl->done)) return;

    // 2. per-column state in LDS: staged source data, g kk in FP64 and FP32
    //    (scalars are loaded only now, so they hold no registers while the
    //    first loads are in flight)
    const double kk = A.prm->kk, eps = A.prm->eps;
    const float kk32 = (float)kk;
    const int has_prev = A.prev_ctl ? A.prev_ctl->has_prev : A.has_prev;
    __syncthreads();  // LDS may still be read by this workgroup's previous job
    src.stage(sm, J);
    double* gs64 = sm + Src::kStageDoubles * ncols;
    float* gs32 = reinterpret_cast<float*>(gs64 + ncols);
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        const double v = (c < J) ? A.g_in[c] * kk : -pinf64();
        gs64[c] = v;
        gs32[c] = (float)v;
    }
    __syncthreads();

    using E = typename std::conditional<P64, double, float>::type;
    E acc[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[ch][v] = 0;
    double res = 0.0;

    // Deferred row outputs (f_i and the residual term) need only (m_i, S_i):
    // lane L keeps those of the wave's L-th row since the last flush, and a
    // flush finishes up to 64 rows at once, so the FP64 logarithms run once
    // per 64 rows instead of once per row.
    double stash_m = 0.0, stash_S = 1.0;
    int64_t stash_i = -1;
    int nstash = 0;
    auto flush = [&]() {
        if (lane < nstash && stash_i < r1) {
            const double ai = A.a[stash_i];
            const double fi = eps * (log(ai) - kLn2 * (stash_m + log2(stash_S)));
            if (has_prev) res += ai * fabs(expm1((A.f_in[stash_i] - fi) / eps));
            A.f_out[stash_i] = fi;
        }
        nstash = 0;
    };

    for (int64_t st0 = 0; step_base(st0) < r1; st0 += RB) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int64_t base = step_base(st0 + q);
            if (base >= r1) break;  // uniform over the wave
            const int64_t i = base + rg;
            const bool vrow = i < r1;
            const int Jl = vrow ? J : 0;
            auto row = src.row(vrow ? i : r0);
            auto cost_at = [&](int ch, int v) -> double {
                const int col = (ch * LPR + sub) * VEC + v;
                if constexpr (Src::kCheap) return src.template cost<P64, VEC>(row, raw[q][ch], v, i, col, sm);
                else return (col < Jl) ? src.template cost<P64, VEC>(row, raw[q][ch], v, i, col, sm) : pinf64();
            };
            E ev[NCH][VEC];
            double m = 0.0, S = 0.0;
            if constexpr (LSE) {
                // shift, exponentials and row sum; a second attempt with the
                // maximum only when the log-sum-exp shift was used and a valid
                // row sum left its range (costs are re-read: LSE sources are cheap)
                static_assert(Src::kCheap, "the log-sum-exp shift re-reads its costs");
                bool by_lse = lse_ok && has_prev;
                for (;;) {
                    if (by_lse) {
                        m = fma(lq[q], kLog2e, -kk * fq[q]);
                    } else {
                        float mx = -__builtin_huge_valf();
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
                            if (ch < nch)
#pragma unroll
                                for (int v = 0; v < VEC; ++v)
                                    mx = fmaxf(mx, fmaf((float)cost_at(ch, v), -kk32, gs32[(ch * LPR + sub) * VEC + v]));
                        m = fmax((double)group_max<LPR>(mx), -1e300);
                    }
                    E s = 0;
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch)
                        if (ch < nch)
#pragma unroll
                            for (int v = 0; v < VEC; ++v) {
                                const double t = fma(cost_at(ch, v), -kk, gs64[(ch * LPR + sub) * VEC + v]) - m;
                                const E e = exp2_f32((float)t);
                                ev[ch][v] = e;
                                s += e;
                            }
                    S = group_sum<LPR>((double)s);
                    if (!by_lse || !__any(vrow && !(S >= 0x1p-100 && S <= 0x1p100))) break;
                    by_lse = false;
                }
            }
            E s_row = 0;
            if constexpr (!LSE) {
                // pass 1: row maximum, an FP32 estimate (it only sets the shift)
                E ck[Src::kCheap ? 1 : NCH][Src::kCheap ? 1 : VEC];
                float mx = -__builtin_huge_valf();
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch)
                    if (ch < nch)
#pragma unroll
                        for (int v = 0; v < VEC; ++v) {
                            const double c = cost_at(ch, v);
                            if constexpr (!Src::kCheap) ck[ch][v] = (E)c;  // exact: the functor's own precision
                            mx = fmaxf(mx, fmaf((float)c, -kk32, gs32[(ch * LPR + sub) * VEC + v]));
                        }
                // (an all-masked row has max -inf: shift by 0 so its terms are 0)
                m = fmax((double)group_max<LPR>(mx), -1e300);
                // pass 2: exponentials (arguments in FP64) and the row sum
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch)
                    if (ch < nch)
#pragma unroll
                        for (int v = 0; v < VEC; ++v) {
                            const double c = Src::kCheap ? cost_at(ch, v) : (double)ck[Src::kCheap ? 0 : ch][Src::kCheap ? 0 : v];
                            const double t = fma(c, -kk, gs64[(ch * LPR + sub) * VEC + v]) - m;
                            E e;
                            if constexpr (P64) e = exp2(t);
                            else e = exp2_f32((float)t);
                            ev[ch][v] = e;
                            s_row += e;
                        }
            }
            const double ai = aq[q];
            // slot q is free: load its rows of the next batch
            issue(q, step_base(st0 + q + RB) + rg);
            if constexpr (!LSE) S = group_sum<LPR>((double)s_row);
            // column partials of the half-iterate plan, pi_ij = e_ij a_i / S_i
            E wq = 0;
            if (vrow) {
                if constexpr (P64) wq = ai / S;
                else wq = (float)ai / (float)S;
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[ch][v] = fma(ev[ch][v], wq, acc[ch][v]);
            // hand (m, S, i) of each row group to lane nstash + r
            const int src_lane = (lane - nstash) * LPR;
            const int sl = (src_lane < 0 || src_lane >= kWave) ? 0 : src_lane;
            const double mm = __shfl(m, sl, kWave);
            const double ss = __shfl(S, sl, kWave);
            if (lane >= nstash && lane < nstash + R) {
                stash_m = mm;
                stash_S = ss;
                stash_i = base + (lane - nstash);
            }
            nstash += R;
            if (nstash == kWave) flush();
        }
    }
    flush();
    res = wave_sum(res);

    // 3. the workgroup's column partials: every (wave, row group) writes its
    //    partial row to LDS once; then each thread sums whole columns over the
    //    WAVES * R contributors in a fixed order, in FP64, and writes them out
    __syncthreads();  // LDS is reused from here on
    E* red = reinterpret_cast<E*>(sm);
    const int contrib = w * R + rg;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        if (ch < nch)
#pragma unroll
            for (int v = 0; v < VEC; ++v) red[contrib * ncols + (ch * LPR + sub) * VEC + v] = acc[ch][v];
    __shared__ double wres[WAVES];
    if (lane == 0) wres[w] = res;
    __syncthreads();
    // (output addresses are formed only here: live registers are scarce)
    double* out = A.col_part + (int64_t)A.part * J;
    for (int c = threadIdx.x; c < J; c += blockDim.x) {
        double t = 0.0;
#pragma unroll 8
        for (int k = 0; k < WAVES * R; ++k) t += (double)red[k * ncols + c];
        out[c] = t;
    }
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int q = 0; q < WAVES; ++q) r += wres[q];
        A.res_part[A.part] = r;
    }
}

// Occupancy the register allocator is asked to keep (waves per SIMD): the
// FP32-exponential dense sweeps with at most 16 columns per lane fit in 128
// registers (4 waves per SIMD) without spills; left to itself the allocator
// sometimes settles a little above 128 and loses a quarter of the occupancy.
template <class Src, bool P64, int VEC, int NCH, int RB>
constexpr int sweep_waves_per_eu() { return (!P64 && Src::kTag == 1 && NCH * RB * VEC <= 16) ? 4 : 1; }

// One Sinkhorn sweep of a single instance: workgroup b owns rows
// [b rows_per_block, (b + 1) rows_per_block).
template <class Src, bool P64, int VEC, int NCH, int LPR, int WAVES, int RB>
__global__ __launch_bounds__(WAVES * kWave)
__attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<Src, P64, VEC, NCH, RB>(), 8))) void k_iter(IterArgs A, Src src) {
    SweepJob job;
    job.r0 = (int64_t)blockIdx.x * A.rows_per_block;
    job.r1 = min(A.I, job.r0 + A.rows_per_block);
    job.J = A.J;
    job.nch = A.nch;
    job.has_prev = 0;
    job.prev_ctl = A.ctl;
    job.prm = A.prm;
    job.a = A.a;
    job.la = A.la;
    job.f_in = A.f_in;
    job.f_out = A.f_out;
    job.g_in = A.g_in;
    job.col_part = A.col_part;
    job.res_part = A.res_part;
    job.part = blockIdx.x;
    sweep_rows<Src, P64, VEC, NCH, LPR, WAVES, RB, !P64 && Src::kCheap>(job, src, A.ctl);
}

// -------------------------------------------------------- column combine --
struct ColArgs {
    int J;
    int nb;  // partial rows
    const double* b;
    const double* g_in;
    double* g_out;
    const double* col_part;
    const double* res_part;
    Ctl* ctl;
    const SolveParams* prm;
    int mode;
    double stall_below;  // fast mode: residuals below this may be declared stalled
};

// Workgroup of 1024 threads = 64 row-lanes x 16 columns: thread (r, c) sums
// partial rows r, r + 64, ... of column c; the 64 row-lanes are then summed
// in a fixed order. Workgroup 0 also closes the iteration's bookkeeping.
constexpr int kColsPerWg = 16;
static __global__ __launch_bounds__(1024) void k_colsum(ColArgs A) {
    Ctl* ctl = A.ctl;
    if (ctl->stop | ctl->done) return;
    const int c = threadIdx.x % kColsPerWg, r = threadIdx.x / kColsPerWg;
    const int j = blockIdx.x * kColsPerWg + c;
    double s = 0.0;
    if (j < A.J) {
        int q = r;
        for (; q + 3 * 64 < A.nb; q += 4 * 64) {
            const double x0 = A.col_part[(int64_t)q * A.J + j], x1 = A.col_part[(int64_t)(q + 64) * A.J + j];
            const double x2 = A.col_part[(int64_t)(q + 128) * A.J + j], x3 = A.col_part[(int64_t)(q + 192) * A.J + j];
            s += x0; s += x1; s += x2; s += x3;
        }
        for (; q < A.nb; q += 64) s += A.col_part[(int64_t)q * A.J + j];
    }
    __shared__ double red[64][kColsPerWg + 1];
    __shared__ int s_bad;
    red[r][c] = s;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if (threadIdx.x < kColsPerWg && j < A.J) {
        double cs = 0.0;
        for (int q = 0; q < 64; ++q) cs += red[q][c];
        const double gn = A.g_in[j] + A.prm->eps * (log(A.b[j]) - log(cs));
        if (!isfinite(gn)) s_bad = 1;
        A.g_out[j] = gn;
    }
    if (blockIdx.x != 0) {
        __syncthreads();
        if (threadIdx.x == 0 && s_bad) ctl->numeric_bad = 1;  // read by the next launch
        return;
    }
    // workgroup 0: total row residual of iterate k-1, then the stop decision
    __shared__ double wr[16];
    double rr = 0.0;
    for (int q = threadIdx.x; q < A.nb; q += blockDim.x) rr += A.res_part[q];
    rr = wave_sum(rr);
    if ((threadIdx.x & 63) == 0) wr[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += wr[q];
        if (s_bad) ctl->numeric_bad = 1;
        bookkeep(ctl, tot, A.mode, A.stall_below);
    }
}

// ------------------------------------------------------------ exact check --
// Statistics of the iterate (f, g) in FP64: row sums, column sums, <C, pi>,
// sum pi (log pi - 1), sum pi and <f, a>, combined in two fixed-order levels
// like k_iter. The last workgroup writes the results into the control block.
struct CheckArgs {
    int64_t I;
    int J;
    int nch;
    int64_t rows_per_block;
    const double* a;
    const double* f;
    const double* g;
    double* col_part;   // gridDim.x x J
    double* stat_part;  // gridDim.x x 5
    const SolveParams* prm;
    double* load_part;  // gridDim.x x J partial RRH loads (the instantiation with loads only)
    void* plan_out;     // I x J row-major plan, FP32 or FP64 (the instantiations with a plan only)
    int plan_f64;
};

// The exact statistics of rows [r0, r1) by one workgroup (one wavefront per
// row): column partials of pi and the five row statistics; with LOADS also
// the column partials of c_ij pi_ij, the RRH loads of Sec. II-B, from the same
// cells (so the loads of the returned plan need no pass of their own); with
// PlanT float or double it also writes each pi_ij it computes, in that type,
// to the row-major plan (so a plan asked for before the solve needs no pass
// of its own either).
struct CheckJob {
    int64_t r0, r1;
    int J;
    int nch;
    double kk;
    const double* a;
    const double* f;
    const double* g;
    double* col_out;   // J
    double* stat_out;  // 5
    double* load_out = nullptr;  // J: sum_i c_ij pi_ij of the rows (with LOADS)
    void* plan_out = nullptr;    // I x J row-major plan of PlanT (with PlanT not void)
};

// Stores VEC consecutive plan values of one lane: as 16-byte (or 8-byte)
// vector stores when `whole` (the VEC columns lie below J and the address is
// aligned to the vector), else one by one for the columns below J.
template <typename T, int VEC>
__device__ __forceinline__ void store_plan(T* dst, const T (&v)[VEC], bool whole, int nvalid) {
    if (whole) {
        if constexpr (sizeof(T) == 4 && VEC == 4) {
            *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
            return;
        } else if constexpr (sizeof(T) == 4 && VEC == 2) {
            *reinterpret_cast<float2*>(dst) = make_float2(v[0], v[1]);
            return;
        } else if constexpr (sizeof(T) == 8 && VEC == 4) {
            reinterpret_cast<double2*>(dst)[0] = make_double2(v[0], v[1]);
            reinterpret_cast<double2*>(dst)[1] = make_double2(v[2], v[3]);
            return;
        } else if constexpr (sizeof(T) == 8 && VEC == 2) {
            *reinterpret_cast<double2*>(dst) = make_double2(v[0], v[1]);
            return;
        }
    }
#pragma unroll
    for (int q = 0; q < VEC; ++q)
        if (q < nvalid) dst[q] = v[q];
}

// True when rows of J values of T starting at `base` keep every lane's VEC
// values aligned to the vector store of store_plan.
template <typename T, int VEC>
__device__ __forceinline__ bool plan_rows_aligned(const void* base, int J) {
    constexpr int a = (int)sizeof(T) * VEC >= 16 ? 16 : (int)sizeof(T) * VEC;
    return J % VEC == 0 && (reinterpret_cast<uintptr_t>(base) % (uintptr_t)a) == 0;
}

template <class Src, int VEC, int NCH, int WAVES, bool LOADS = false, typename PlanT = void>
__device__ __forceinline__ void check_rows(const CheckJob& A, const Src& src) {
    constexpr bool kPlan = !std::is_void<PlanT>::value;
    extern __shared__ double sm[];
    const double kk = A.kk;
    const int J = A.J, nch = A.nch;
    const int ncols = nch * kWave * VEC;
    __syncthreads();  // LDS may still be read by this workgroup's previous job
    src.stage(sm, J);
    __shared__ double e2tab[64];
    exp2_tab_fill(e2tab);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double gsr[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int col = (ch * kWave + lane) * VEC + v;
            gsr[ch][v] = (ch < nch && col < J) ? A.g[col] * kk : -pinf64();
        }
    __syncthreads();
    double acc[NCH][VEC], accl[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[ch][v] = accl[ch][v] = 0.0;
    double st[5] = {0, 0, 0, 0, 0};  // rowres, cost, ent, mass, fa (lane 0 of each wave)
    double cost = 0.0, ent = 0.0;     // this lane's cells of <C, pi> and sum pi (log pi - 1)
    bool plan_vec = false;            // the plan's rows take vector stores
    if constexpr (kPlan) plan_vec = plan_rows_aligned<PlanT, VEC>(A.plan_out, J);
    // The loads of a row (its costs, f_i and a_i) are issued one row ahead,
    // so that a wave waits for memory only when a row's arithmetic is shorter
    // than the load latency.
    typename Src::template Raw<VEC> nraw[NCH];
    double nf = 0.0, na = 0.0;
    auto fetch = [&](int64_t i) {
        auto row = src.row(i);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (ch < nch) nraw[ch] = src.template load<VEC>(row, (ch * kWave + lane) * VEC, J);
        nf = A.f[i];
        na = A.a[i];
    };
    if (A.r0 + w < A.r1) fetch(A.r0 + w);
    for (int64_t i = A.r0 + w; i < A.r1; i += WAVES) {
        typename Src::template Raw<VEC> raw[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) raw[ch] = nraw[ch];
        const double fi = nf, ai = na;
        if (i + WAVES < A.r1) fetch(i + WAVES);
        auto row = src.row(i);
        const double fk = fi * kk;
        double rs = 0.0;
        using PlanS = typename std::conditional<kPlan, PlanT, float>::type;
        PlanS* prow = kPlan ? reinterpret_cast<PlanS*>(A.plan_out) + i * (int64_t)J : nullptr;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            if (ch < nch) {
                const int col0 = (ch * kWave + lane) * VEC;
                PlanS pv[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    // a column past J adds exact zeros (p = 0, c = 0), which
                    // leaves every sum as it was
                    const bool ok = col0 + v < J;
                    const double c = ok ? src.template cost<true, VEC>(row, raw[ch], v, i, ok ? col0 + v : J - 1, sm) : 0.0;
                    const double t = ok ? fk + fma(c, -kk, gsr[ch][v]) : 0.0;  // log2 pi_ij
                    const double e = exp2_tab(t, e2tab);  // (t = 0 where !ok: no branch)
                    const double p = ok ? e : 0.0;
                    rs += p;
                    cost = fma(c, p, cost);
                    ent = fma(p, t * kLn2 - 1.0, ent);
                    acc[ch][v] += p;
                    if constexpr (LOADS) accl[ch][v] = fma(c, p, accl[ch][v]);
                    pv[v] = (PlanS)p;
                }
                if constexpr (kPlan) store_plan<PlanS, VEC>(prow + col0, pv, plan_vec && col0 + VEC <= J, J - col0);
            }
        }
        rs = wave_sum(rs);
        if (lane == 0) {
            st[0] += fabs(rs - ai);
            st[3] += rs;
            st[4] += fi * ai;
        }
    }
    // <C, pi> and the entropy term need no per-row total: each lane sums its
    // cells over the wave's rows, and the wave folds them once
    {
        const double tc = wave_sum(cost), te = wave_sum(ent);
        if (lane == 0) {
            st[1] = tc;
            st[2] = te;
        }
    }
    __syncthreads();
    __shared__ double wst[WAVES][5];
    if (lane == 0)
        for (int q = 0; q < 5; ++q) wst[w][q] = st[q];
    block_tree<NCH, VEC, WAVES>(acc, nch, sm, ncols, w, lane);
    if (w == 0) {
        double* out = A.col_out;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (ch < nch)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const int col = (ch * kWave + lane) * VEC + v;
                    if (col < J) out[col] = acc[ch][v];
                }
        if (lane < 5) {
            double r = 0.0;
            for (int q = 0; q < WAVES; ++q) r += wst[q][lane];
            A.stat_out[lane] = r;
        }
    }
    if constexpr (LOADS) {
        // (the tree above ended on a barrier and wave 0 has not touched the
        // LDS since, so the second tree can start at once)
        block_tree<NCH, VEC, WAVES>(accl, nch, sm, ncols, w, lane);
        if (w == 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        const int col = (ch * kWave + lane) * VEC + v;
                        if (col < J) A.load_out[col] = accl[ch][v];
                    }
        }
    }
}

// The same check with the lane layout of the sweeps: LPR (16 or 32) lanes
// per row, R = 64 / LPR rows per wave step, lane `sub` owning columns
// (ch LPR + sub) VEC + v. For short rows (tens of RRHs) this keeps the lanes
// busy where one row per wavefront would leave most of them idle. Every sum
// runs in a fixed order.
template <class Src, int VEC, int NCH, int LPR, int WAVES>
__device__ __forceinline__ void check_rows_g(const CheckJob& A, const Src& src) {
    extern __shared__ double sm[];
    constexpr int R = kWave / LPR;
    const double kk = A.kk;
    const int J = A.J, nch = A.nch;
    const int ncols = nch * LPR * VEC;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int sub = lane % LPR, rg = lane / LPR;
    __syncthreads();  // LDS may still be read by this workgroup's previous job
    src.stage(sm, J);
    __shared__ double e2tab[64];
    exp2_tab_fill(e2tab);
    double gsr[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int col = (ch * LPR + sub) * VEC + v;
            gsr[ch][v] = (ch < nch && col < J) ? A.g[col] * kk : -pinf64();
        }
    __syncthreads();
    double acc[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[ch][v] = 0.0;
    double st[5] = {0, 0, 0, 0, 0};  // rowres, cost, ent, mass, fa (first lane of each row group)
    for (int64_t base = A.r0 + (int64_t)w * R; base < A.r1; base += (int64_t)WAVES * R) {
        const int64_t i = base + rg;
        const bool vrow = i < A.r1;
        auto row = src.row(vrow ? i : A.r0);
        const double fi = vrow ? A.f[i] : 0.0;
        const double fk = fi * kk;
        double rs = 0.0, cost = 0.0, ent = 0.0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            if (ch < nch) {
                const int col0 = (ch * LPR + sub) * VEC;
                double c[VEC];
                src.template get<true, VEC>(row, i, col0, vrow ? J : 0, sm, c);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    // a row or column outside the job adds exact zeros (p = 0,
                    // c = 0), which leaves every sum as it was
                    const bool ok = vrow && col0 + v < J;
                    const double cv = ok ? c[v] : 0.0;
                    const double t = ok ? fk + fma(cv, -kk, gsr[ch][v]) : 0.0;  // log2 pi_ij
                    const double e = exp2_tab(t, e2tab);
                    const double p = ok ? e : 0.0;
                    rs += p;
                    cost = fma(cv, p, cost);
                    ent = fma(p, t * kLn2 - 1.0, ent);
                    acc[ch][v] += p;
                }
            }
        }
        rs = group_sum<LPR>(rs);
        cost = group_sum<LPR>(cost);
        ent = group_sum<LPR>(ent);
        if (sub == 0 && vrow) {
            const double ai = A.a[i];
            st[0] += fabs(rs - ai);
            st[1] += cost;
            st[2] += ent;
            st[3] += rs;
            st[4] += fi * ai;
        }
    }
    // the row groups of a wave share columns: fold them, then the waves
#pragma unroll
    for (int o = LPR; o < kWave; o <<= 1)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[ch][v] += __shfl_xor(acc[ch][v], o, kWave);
#pragma unroll
    for (int q = 0; q < 5; ++q) st[q] = wave_sum(st[q]);
    __syncthreads();
    double* red = sm;
#pragma unroll
    for (int half = WAVES / 2; half >= 1; half >>= 1) {
        if (w >= half && w < 2 * half && rg == 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) red[(w - half) * ncols + (ch * LPR + sub) * VEC + v] = acc[ch][v];
        }
        __syncthreads();
        if (w < half && rg == 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[ch][v] += red[w * ncols + (ch * LPR + sub) * VEC + v];
        }
        __syncthreads();
    }
    __shared__ double wst[WAVES][5];
    if (lane == 0)
        for (int q = 0; q < 5; ++q) wst[w][q] = st[q];
    __syncthreads();
    if (w == 0) {
        if (rg == 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch < nch)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        const int col = (ch * LPR + sub) * VEC + v;
                        if (col < J) A.col_out[col] = acc[ch][v];
                    }
        }
        if (lane < 5) {
            double r = 0.0;
            for (int q = 0; q < WAVES; ++q) r += wst[q][lane];
            A.stat_out[lane] = r;
        }
    }
}

template <class Src, int VEC, int NCH, int WAVES, bool LOADS = false, typename PlanT = void>
__global__ __launch_bounds__(WAVES * kWave) void k_check(CheckArgs A, Src src) {
    CheckJob job;
    job.r0 = (int64_t)blockIdx.x * A.rows_per_block;
    job.r1 = min(A.I, job.r0 + A.rows_per_block);
    job.J = A.J;
    job.nch = A.nch;
    job.kk = A.prm->kk;
    job.a = A.a;
    job.f = A.f;
    job.g = A.g;
    job.col_out = A.col_part + (int64_t)blockIdx.x * A.J;
    job.stat_out = A.stat_part + (int64_t)blockIdx.x * 5;
    if constexpr (LOADS) job.load_out = A.load_part + (int64_t)blockIdx.x * A.J;
    job.plan_out = A.plan_out;
    check_rows<Src, VEC, NCH, WAVES, LOADS, PlanT>(job, src);
}

// Column sums of the check: per column |colsum_j - b_j| and g_j b_j, summed
// per workgroup of 16 columns (same layout as k_colsum); with load partials
// also each RRH's load, their fixed-order column sum.
struct CheckColArgs {
    int J;
    int nb;
    const double* b;
    const double* g;
    const double* col_part;
    double* cpart;            // gridDim.x x 2
    const double* load_part;  // nb x J, or null
    double* loads;            // J (with load_part)
};

static __global__ __launch_bounds__(1024) void k_check_cols(CheckColArgs A) {
    static_assert(kColsPerWg * 64 == 1024, "64 partial sums per column");
    const int c = threadIdx.x % kColsPerWg, r = threadIdx.x / kColsPerWg;
    const int j = blockIdx.x * kColsPerWg + c;
    // (eight loads in flight, added in index order)
    auto fold = [&](const double* part) {
        double s = 0.0;
        int q = r;
        for (; q + 7 * 64 < A.nb; q += 8 * 64) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(q + u * 64) * A.J + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; q < A.nb; q += 64) s += part[(int64_t)q * A.J + j];
        return s;
    };
    const bool with_loads = A.load_part != nullptr;
    __shared__ double red[64][kColsPerWg + 1];
    __shared__ double redl[64][kColsPerWg + 1];
    __shared__ double colres[kColsPerWg][2];
    red[r][c] = j < A.J ? fold(A.col_part) : 0.0;
    if (with_loads) redl[r][c] = j < A.J ? fold(A.load_part) : 0.0;
    __syncthreads();
    // one thread per column folds its 64 partials in order, then thread 0
    // takes the columns in order
    if (threadIdx.x < kColsPerWg) {
        const int jj = blockIdx.x * kColsPerWg + threadIdx.x;
        double cs = 0.0;
        for (int q = 0; q < 64; ++q) cs += red[q][threadIdx.x];
        colres[threadIdx.x][0] = jj < A.J ? fabs(cs - A.b[jj]) : 0.0;
        colres[threadIdx.x][1] = jj < A.J ? A.g[jj] * A.b[jj] : 0.0;
        if (with_loads && jj < A.J) {
            double ls = 0.0;
            for (int q = 0; q < 64; ++q) ls += redl[q][threadIdx.x];
            A.loads[jj] = ls;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double cres = 0.0, gb = 0.0;
        for (int cc = 0; cc < kColsPerWg; ++cc) {
            if (blockIdx.x * kColsPerWg + cc >= A.J) break;
            cres += colres[cc][0];
            gb += colres[cc][1];
        }
        A.cpart[blockIdx.x * 2] = cres;
        A.cpart[blockIdx.x * 2 + 1] = gb;
    }
}

// One workgroup: the check's scalars, in a fixed order, into the control block.
static __global__ __launch_bounds__(256) void k_check_finish(const double* stat_part, int nb, const double* cpart, int ncb,
                                                      Ctl* ctl, const SolveParams* prm) {
    __shared__ double red[4][7];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < nb; q += blockDim.x)
        for (int u = 0; u < 5; ++u) v[u] += stat_part[(int64_t)q * 5 + u];
    for (int q = threadIdx.x; q < ncb; q += blockDim.x) { v[5] += cpart[q * 2]; v[6] += cpart[q * 2 + 1]; }
    for (int u = 0; u < 7; ++u) {
        v[u] = wave_sum(v[u]);
        if (lane == 0) red[w][u] = v[u];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[7];
        for (int u = 0; u < 7; ++u) t[u] = ((red[0][u] + red[1][u]) + red[2][u]) + red[3][u];
        const double eps = prm->eps;
        ctl->chk_row_res = t[0];
        ctl->chk_col_res = t[5];
        ctl->chk_violation = (t[0] + t[5]) / ctl->mass;
        ctl->chk_objective = t[1];
        ctl->chk_reg_objective = t[1] + eps * t[2];
        ctl->chk_mass = t[3];
        ctl->chk_dual = t[4] + t[6] - eps * t[3];
    }
}

// -------------------------------------------------------------------- plan --
// pi_ij = exp((f_i + g_j - C_ij) / eps) in FP64, stored as OutT.
// Rows [r0, r1); `out` holds row r0 first.
template <class Src, typename OutT, int VEC>
__global__ __launch_bounds__(512) void k_plan(int64_t r0, int64_t r1, int J, int nch, const double* f, const double* g,
                                              const SolveParams* prm, OutT* out, Src src) {
    const double kk = prm->kk;
    const int ncols = nch * kWave * VEC;
    extern __shared__ double sm[];
    double* stage = sm;
    double* gs = sm + Src::kStageDoubles * ncols;
    src.stage(stage, J);
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) gs[c] = (c < J) ? g[c] * kk : -pinf64();
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    for (int64_t i = r0 + (int64_t)blockIdx.x * nw + w; i < r1; i += (int64_t)gridDim.x * nw) {
        auto row = src.row(i);
        const double fk = f[i] * kk;
        OutT* o = out + (i - r0) * J;
        for (int ch = 0; ch < nch; ++ch) {
            const int col0 = (ch * kWave + lane) * VEC;
            double c[VEC];
            src.template get<true, VEC>(row, i, col0, J, stage, c);
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (col0 + v < J) o[col0 + v] = (OutT)exp2(fk + fma(c[v], -kk, gs[col0 + v]));
        }
    }
}

// ------------------------------------------------------------- validation --
// Flags a non-finite dense cost, or a rate that is not finite and positive:
// ORs `bit` into *bad and, when ctl is given, ends the solve on the device
// (done and stop) so that a solve needs no host round trip for the check.
template <typename T, bool RATES>
__global__ void k_validate(const T* x, int64_t I, int J, int64_t ld, int* bad, int bit, Ctl* ctl) {
    int flag = 0;
    const int64_t n = I * J;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / J;
        const double v = (double)x[i * ld + (q - i * J)];
        if (RATES ? !(v > 0.0 && isfinite(v)) : !isfinite(v)) flag = 1;
    }
    if (__any(flag) && (threadIdx.x & 63) == 0) {
        atomicOr(bad, bit);
        if (ctl) {
            ctl->done = 1;
            ctl->stop = 1;
        }
    }
}

static __global__ void k_validate_xy(const float* xy, int64_t n, int* bad, int bit, Ctl* ctl) {
    int flag = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(xy[q])) flag = 1;
    if (__any(flag) && (threadIdx.x & 63) == 0) {
        atomicOr(bad, bit);
        if (ctl) {
            ctl->done = 1;
            ctl->stop = 1;
        }
    }
}

// Clears the stop flag between phases (kept as a kernel so that it may sit in
// a captured graph).
static __global__ void k_ctl_resume(Ctl* ctl) {
    if (threadIdx.x == 0) ctl->stop = 0;
}

}  // namespace otk
