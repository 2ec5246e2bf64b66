// Kernels of the batched engine: many independent association instances
// advance together, one Sinkhorn iteration per group of three launches.
//
// Every instance carries its own phase in its control block:
//   fast    FP32-exponential sweeps until the residual meets tol or stalls;
//   polish  a fixed number of FP64 sweeps;
//   check   the exact FP64 statistics of one iterate (no new iterate);
//   exact   FP64 sweeps until an FP64 iterate meets tol (only when a check
//           misses tol), then the check again;
//   done.
// Work is described by device-side lists that the combine kernel of each
// iteration rebuilds for the next: a sweep list of (instance, row part) items
// in FP32, one in FP64 (sweeps and checks), and the list of instances whose
// columns must be combined. The sweep kernels are persistent (a grid that
// fills the GPU once, each workgroup walking the list with a stride), so a
// captured chunk of iterations never depends on how many instances or parts
// are live. Every item writes its own partial rows; all sums run in a fixed
// order, so an instance's result does not depend on its neighbours in the
// batch or on which workgroup ran which item.
#pragma once

#include "kernels.h"

namespace otk {

constexpr int kBatchMaxJ = 512;  // RRHs per batched instance (4 column classes)

enum : int { kPhFast = 0, kPhPolish = 1, kPhCheck = 2, kPhExact = 3, kPhDone = 4 };
enum : int { kItPrev = 1, kItPar = 2, kItCheck = 4 };

// One instance of the batch. The cost is a padded FP32 row-major matrix
// (row stride ld, a multiple of 4 floats, padding +inf).
struct BInst {
    const float* C;
    int64_t ld;
    int64_t I;
    int J;
    int cls;     // lane / column-chunk class of the sweeps
    int nch;     // column chunks of the sweeps
    int nchk;    // column chunks of the 64-lane check
    int parts;   // row parts (items) of every sweep
    int pad_;
    int64_t rpp;  // rows per part
    const double* a;
    const double* b;
    double* f[2];
    double* g[2];
    double* col_part;   // parts x J
    double* res_part;   // parts
    double* stat_part;  // parts x 5
    Ctl* ctl;
    double kk, eps;
};

struct BItem {
    int inst, part, flags, pad_;
};

// One generation of work lists; cnt[0] FP32 items, cnt[1] FP64 items,
// cnt[2] instances to combine.
struct BList {
    BItem* it32;
    BItem* it64;
    int* inst;
    int* cnt;
};

struct BParams {
    int polish_iters;
    double stall_below;
};

// Column classes: (lanes per row, column chunks of 4 FP32 values per lane).
__host__ __device__ constexpr int batch_class(int J) { return J <= 64 ? 0 : J <= 128 ? 1 : J <= 256 ? 2 : 3; }
__host__ __device__ constexpr int batch_class_lpr(int cls) { return cls == 3 ? 32 : 16; }
__host__ __device__ constexpr int batch_class_nch(int cls) { return cls == 0 ? 1 : cls == 1 ? 2 : 4; }

template <bool P64, int WAVES>
__device__ __forceinline__ void batch_sweep_item(const BInst& d, const BItem& it, double* sm) {
    const int pin = (it.flags & kItPar) ? 1 : 0;
    SweepJob job;
    job.r0 = (int64_t)it.part * d.rpp;
    job.r1 = min(d.I, job.r0 + d.rpp);
    job.J = d.J;
    job.nch = d.nch;
    job.has_prev = (it.flags & kItPrev) ? 1 : 0;
    job.kk = d.kk;
    job.eps = d.eps;
    job.a = d.a;
    job.f_in = d.f[pin];
    job.f_out = d.f[pin ^ 1];
    job.g_in = d.g[pin];
    job.col_out = d.col_part + (int64_t)it.part * d.J;
    job.res_out = d.res_part + it.part;
    const DenseSrc<float> src{d.C, d.ld};
    using S = DenseSrc<float>;
    switch (d.cls) {
        case 0: sweep_rows<S, P64, 4, 1, 16, WAVES, 1>(job, src, sm, nullptr); break;
        case 1: sweep_rows<S, P64, 4, 2, 16, WAVES, 1>(job, src, sm, nullptr); break;
        case 2: sweep_rows<S, P64, 4, 4, 16, WAVES, 1>(job, src, sm, nullptr); break;
        default: sweep_rows<S, P64, 4, 4, 32, WAVES, 1>(job, src, sm, nullptr); break;
    }
}

// Persistent sweep over the FP32 (P64 = false) or FP64 (P64 = true) list.
// The FP32 kernel also clears the counters of the next generation, which
// nothing reads or writes before the combine kernel of this iteration.
template <bool P64, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_bsweep(const BInst* tab, BList in, BList out) {
    extern __shared__ double sm[];
    if (!P64 && blockIdx.x == 0 && threadIdx.x < 3) out.cnt[threadIdx.x] = 0;
    const int n = in.cnt[P64 ? 1 : 0];
    const BItem* items = P64 ? in.it64 : in.it32;
    for (int q = blockIdx.x; q < n; q += gridDim.x) {
        const BItem it = items[q];
        const BInst& d = tab[it.inst];
        if constexpr (P64) {
            if (it.flags & kItCheck) {
                const int par = (it.flags & kItPar) ? 1 : 0;
                CheckJob cj;
                cj.r0 = (int64_t)it.part * d.rpp;
                cj.r1 = min(d.I, cj.r0 + d.rpp);
                cj.J = d.J;
                cj.nch = d.nchk;
                cj.kk = d.kk;
                cj.a = d.a;
                cj.f = d.f[par];
                cj.g = d.g[par];
                cj.col_out = d.col_part + (int64_t)it.part * d.J;
                cj.stat_out = d.stat_part + (int64_t)it.part * 5;
                check_rows<DenseSrc<float>, 4, 2, WAVES>(cj, DenseSrc<float>{d.C, d.ld}, sm);
                continue;
            }
        }
        batch_sweep_item<P64, WAVES>(d, it, sm);
    }
}

// Per instance of the list: the column combine of the sweep (new g) or of the
// check, then the phase machine, then the instance's items of the next
// iteration. One workgroup of 1024 threads = 16 part-lanes x 64 columns.
__global__ __launch_bounds__(1024) void k_bcombine(const BInst* tab, BList in, BList out, BParams P) {
    __shared__ double red[16][65];
    __shared__ double wsum[16][7];
    __shared__ int s_bad, s_list, s_base, s_flags;
    const int n = in.cnt[2];
    const int tid = threadIdx.x, c = tid & 63, r = tid >> 6, lane = tid & 63, w = tid >> 6;
    for (int q = blockIdx.x; q < n; q += gridDim.x) {
        const int k = in.inst[q];
        const BInst& d = tab[k];
        Ctl* ctl = d.ctl;
        const int phase = ctl->phase;
        const bool check = phase == kPhCheck;
        const int J = d.J, parts = d.parts;
        const int pin = check ? (ctl->check_iter & 1) : (ctl->iter & 1);
        if (tid == 0) s_bad = 0;
        __syncthreads();
        // columns, 64 at a time: fixed-order sums over the parts
        double cres = 0.0, gb = 0.0;
        for (int j0 = 0; j0 < J; j0 += 64) {
            const int j = j0 + c;
            double s = 0.0;
            if (j < J)
                for (int p = r; p < parts; p += 16) s += d.col_part[(int64_t)p * J + j];
            red[r][c] = s;
            __syncthreads();
            if (tid < 64 && j < J) {
                double cs = 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) cs += red[u][c];
                if (check) {
                    cres += fabs(cs - d.b[j]);
                    gb += d.g[pin][j] * d.b[j];
                } else {
                    const double gn = d.g[pin][j] + d.eps * (log(d.b[j]) - log(cs));
                    if (!isfinite(gn)) s_bad = 1;
                    d.g[pin ^ 1][j] = gn;
                }
            }
            __syncthreads();
        }
        // per-part scalars: the row residual, or the check's five statistics
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        if (check) {
            for (int p = tid; p < parts; p += 1024)
                for (int u = 0; u < 5; ++u) v[u] += d.stat_part[(int64_t)p * 5 + u];
            v[5] = cres;
            v[6] = gb;
        } else {
            for (int p = tid; p < parts; p += 1024) v[0] += d.res_part[p];
        }
        for (int u = 0; u < 7; ++u) {
            const double t = wave_sum(v[u]);
            if (lane == 0) wsum[w][u] = t;
        }
        __syncthreads();
        if (tid == 0) {
            double t[7];
            for (int u = 0; u < 7; ++u) {
                double x = 0.0;
                for (int q2 = 0; q2 < 16; ++q2) x += wsum[q2][u];
                t[u] = x;
            }
            int next = -1;  // -1 none, 0 FP32 sweep, 1 FP64 sweep, 2 check
            if (check) {
                const double viol = (t[0] + t[5]) / ctl->mass;
                ctl->chk_row_res = t[0];
                ctl->chk_col_res = t[5];
                ctl->chk_violation = viol;
                ctl->chk_objective = t[1];
                ctl->chk_reg_objective = t[1] + d.eps * t[2];
                ctl->chk_mass = t[3];
                ctl->chk_dual = t[4] + t[6] - d.eps * t[3];
                if (viol < ctl->tol || ctl->exact_done || ctl->iter >= ctl->max_iter || !isfinite(viol)) {
                    ctl->phase = kPhDone;
                    ctl->done = 1;
                    ctl->result_iter = ctl->check_iter;
                } else {
                    ctl->phase = kPhExact;
                    next = 1;
                }
            } else {
                const int mode = phase == kPhFast ? kModeFast : phase == kPhPolish ? kModePolish : kModeExact;
                if (s_bad) ctl->numeric_bad = 1;
                bookkeep(ctl, t[0], mode, P.stall_below);
                if (ctl->numeric_bad) {
                    ctl->phase = kPhDone;  // bookkeep has set done and result_iter
                } else if (ctl->done) {
                    // exact phase: an FP64 iterate met tol; check that iterate
                    ctl->done = 0;
                    ctl->phase = kPhCheck;
                    ctl->check_iter = ctl->result_iter;
                    ctl->exact_done = 1;
                    next = 2;
                } else if (ctl->stop) {
                    ctl->stop = 0;
                    if (phase == kPhFast && P.polish_iters > 0 && ctl->iter < ctl->max_iter) {
                        ctl->phase = kPhPolish;
                        ctl->polish_left = P.polish_iters;
                        next = 1;
                    } else {
                        if (phase != kPhFast) ctl->exact_done = 1;  // the iteration cap was reached
                        ctl->phase = kPhCheck;
                        ctl->check_iter = ctl->iter;
                        next = 2;
                    }
                } else if (phase == kPhPolish) {
                    if (--ctl->polish_left <= 0) {
                        ctl->phase = kPhCheck;
                        ctl->check_iter = ctl->iter;
                        next = 2;
                    } else {
                        next = 1;
                    }
                } else {
                    next = phase == kPhFast ? 0 : 1;
                }
            }
            s_list = next;
            if (next >= 0) {
                const int par = (next == 2 ? ctl->check_iter : ctl->iter) & 1;
                s_flags = (ctl->has_prev ? kItPrev : 0) | (par ? kItPar : 0) | (next == 2 ? kItCheck : 0);
                s_base = atomicAdd(&out.cnt[next == 0 ? 0 : 1], parts);
                out.inst[atomicAdd(&out.cnt[2], 1)] = k;
            }
        }
        __syncthreads();
        if (s_list >= 0) {
            BItem* dst = (s_list == 0 ? out.it32 : out.it64) + s_base;
            for (int p = tid; p < parts; p += 1024) dst[p] = BItem{k, p, s_flags, 0};
        }
        __syncthreads();  // shared state is rewritten by the next instance
    }
}

// Appends admitted instances (their first FP32 sweep items) to a list
// generation that no kernel is using (stream order puts it between chunks).
__global__ __launch_bounds__(256) void k_badmit(BList l, const BItem* items, int n_items, const int* insts,
                                                 int n_insts) {
    __shared__ int s_bi, s_bk;
    if (threadIdx.x == 0) {
        s_bi = l.cnt[0];
        s_bk = l.cnt[2];
        l.cnt[0] = s_bi + n_items;
        l.cnt[2] = s_bk + n_insts;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_items; q += blockDim.x) l.it32[s_bi + q] = items[q];
    for (int q = threadIdx.x; q < n_insts; q += blockDim.x) l.inst[s_bk + q] = insts[q];
}

// Clears a list generation (all three counters).
__global__ void k_bclear(BList l) {
    if (threadIdx.x < 3) l.cnt[threadIdx.x] = 0;
}

// Padded FP32 copy of a cost source: dst[i ld + j] = cost(i, j) for j < J,
// +inf for J <= j < ld. KIND 0: dense C; 1: rates, c = inv_scale / R.
template <typename T, int KIND>
__global__ void k_bpad(const T* src, int64_t I, int J, int64_t lds, float* dst, int64_t ld, double inv_scale) {
    const int64_t n = I * ld;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ld;
        const int j = (int)(e - i * ld);
        float v = __builtin_huge_valf();
        if (j < J) {
            const double x = (double)src[i * lds + j];
            v = KIND == 0 ? (float)x : (float)((1.0 / x) * inv_scale);
        }
        dst[e] = v;
    }
}

// Non-finite or non-positive entry detection for batch inputs (bad = 1).
template <typename T, bool POS>
__global__ void k_bvalidate(const T* x, int64_t I, int J, int64_t lds, int* bad) {
    const int64_t n = I * J;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / J;
        const double v = (double)x[i * lds + (e - i * J)];
        if (!isfinite(v) || (POS && !(v > 0.0))) *bad = 1;
    }
}

}  // namespace otk
