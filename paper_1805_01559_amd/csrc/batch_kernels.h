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

#include "setup_kernels.h"

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
    const SolveParams* prm;  // kk, eps in device memory
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

// Column classes: (lanes per row, column chunks of 4 FP32 values per lane):
// (16, 1), (16, 2), (16, 4), (32, 4) for J up to 64, 128, 256, 512. The one
// kernel that holds every class stays within the register budget of
// 3 waves per SIMD.
__host__ __device__ constexpr int batch_class(int J) { return J <= 64 ? 0 : J <= 128 ? 1 : J <= 256 ? 2 : 3; }
__host__ __device__ constexpr int batch_class_lpr(int cls) { return cls == 3 ? 32 : 16; }
__host__ __device__ constexpr int batch_class_nch(int cls) { return cls == 0 ? 1 : cls == 1 ? 2 : 4; }

template <bool P64, int WAVES>
__device__ __forceinline__ void batch_sweep_item(const BInst& d, const BItem& it) {
    const int pin = (it.flags & kItPar) ? 1 : 0;
    SweepJob job;
    job.r0 = (int64_t)it.part * d.rpp;
    job.r1 = min(d.I, job.r0 + d.rpp);
    job.J = d.J;
    job.nch = d.nch;
    job.has_prev = (it.flags & kItPrev) ? 1 : 0;
    job.prev_ctl = nullptr;
    job.prm = d.prm;
    job.a = d.a;
    job.la = nullptr;  // (the batch sweeps shift rows by their maximum)
    job.f_in = d.f[pin];
    job.f_out = d.f[pin ^ 1];
    job.g_in = d.g[pin];
    job.col_part = d.col_part;
    job.res_part = d.res_part;
    job.part = it.part;
    const DenseSrc<float> src{d.C, d.ld};
    using S = DenseSrc<float>;
    switch (d.cls) {
        case 0: sweep_rows<S, P64, 4, 1, 16, WAVES, 1, false>(job, src, nullptr); break;
        case 1: sweep_rows<S, P64, 4, 2, 16, WAVES, 1, false>(job, src, nullptr); break;
        case 2: sweep_rows<S, P64, 4, 4, 16, WAVES, 1, false>(job, src, nullptr); break;
        default: sweep_rows<S, P64, 4, 4, 32, WAVES, 1, false>(job, src, nullptr); break;
    }
}

// Persistent sweep over the FP32 (P64 = false) or FP64 (P64 = true) list.
// The FP32 kernel also clears the counters of the next generation, which
// nothing reads or writes before the combine kernel of this iteration.
// (the table, the list and its counter are read-only here and marked so:
// their uniform loads then go through the scalar unit into SGPRs)
template <bool P64, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_bsweep(const BInst* __restrict__ tab,
                                                          const BItem* __restrict__ items,
                                                          const int* __restrict__ cnt_in, int* __restrict__ cnt_out) {
    if (!P64 && blockIdx.x == 0 && threadIdx.x < 3) cnt_out[threadIdx.x] = 0;
    const int n = cnt_in[P64 ? 1 : 0];
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
                cj.nch = d.nch;
                cj.kk = d.kk;
                cj.a = d.a;
                cj.f = d.f[par];
                cj.g = d.g[par];
                cj.col_out = d.col_part + (int64_t)it.part * d.J;
                cj.stat_out = d.stat_part + (int64_t)it.part * 5;
                const DenseSrc<float> src{d.C, d.ld};
                using S = DenseSrc<float>;
                switch (d.cls) {  // the sweeps' lane layout of the instance's column class
                    case 0: check_rows_g<S, 4, 1, 16, WAVES>(cj, src); break;
                    case 1: check_rows_g<S, 4, 2, 16, WAVES>(cj, src); break;
                    case 2: check_rows_g<S, 4, 4, 16, WAVES>(cj, src); break;
                    default: check_rows_g<S, 4, 4, 32, WAVES>(cj, src); break;
                }
                continue;
            }
        }
        batch_sweep_item<P64, WAVES>(d, it);
    }
}

// Per instance of the list: the column combine of the sweep (new g) or of the
// check, then the phase machine, then the instance's items of the next
// iteration. One workgroup of 1024 threads: thread t takes column
// (t / 64 mod NC2) 64 + t mod 64 of the NC2 = 2^ceil(log2(J / 64)) column
// chunks and part group t / (64 NC2) of the PG = 1024 / (64 NC2) groups; a
// group sums its parts (every PG-th) sixteen loads at a time in a fixed
// tree, and the groups' sums are added in group order, so each column's sum
// has one fixed order for given J and part count.
// An instance still running after kFineIter iterations (the few slow ones
// that remain at the end of a batch) continues in parts of kFineRows rows, so
// that a sweep spreads it over more workgroups when little else runs. The
// switch depends on the instance's own iteration count only, so its result
// does not depend on its neighbours in the batch.
constexpr int kCombLoads = 16;
constexpr int kFineIter = 32;
constexpr int64_t kFineRows = 64;
__global__ __launch_bounds__(1024) void k_bcombine(BInst* tab, BList in, BList out, BParams P) {
    __shared__ double red[1024];
    __shared__ double wsum[16][7];
    __shared__ int s_bad, s_list, s_base, s_flags, s_parts;
    const int n = in.cnt[2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = blockIdx.x; q < n; q += gridDim.x) {
        const int k = in.inst[q];
        const BInst& d = tab[k];
        Ctl* ctl = d.ctl;
        const int phase = ctl->phase;
        if (phase == kPhDone) continue;  // rejected at admission: no work, no next items (uniform)
        const bool check = phase == kPhCheck;
        const int J = d.J, parts = d.parts;
        const int pin = check ? (ctl->check_iter & 1) : (ctl->iter & 1);
        if (tid == 0) s_bad = 0;
        int nc2 = 1;
        while (nc2 * 64 < J) nc2 <<= 1;  // J <= 512: at most 8 chunks
        const int pg = 1024 / (64 * nc2);
        const int grp = tid / (64 * nc2);
        const int j = ((tid >> 6) & (nc2 - 1)) * 64 + lane;
        double s = 0.0;
        if (j < J) {
            const double* cp = d.col_part + j;
            int p = grp;
            for (; p + (kCombLoads - 1) * pg < parts; p += kCombLoads * pg) {
                double x[kCombLoads];
#pragma unroll
                for (int u = 0; u < kCombLoads; ++u) x[u] = cp[(int64_t)(p + u * pg) * J];
#pragma unroll
                for (int h = kCombLoads / 2; h > 0; h >>= 1)
#pragma unroll
                    for (int u = 0; u < h; ++u) x[u] += x[u + h];
                s += x[0];
            }
            for (; p < parts; p += pg) s += cp[(int64_t)p * J];
        }
        red[grp * (64 * nc2) + j] = s;  // (j < 64 nc2: every thread has its own slot)
        __syncthreads();
        double cres = 0.0, gb = 0.0;
        if (tid < J) {
            double cs = 0.0;
            for (int u = 0; u < pg; ++u) cs += red[u * (64 * nc2) + tid];
            if (check) {
                cres = fabs(cs - d.b[tid]);
                gb = d.g[pin][tid] * d.b[tid];
            } else {
                const double gn = d.g[pin][tid] + d.eps * (log(d.b[tid]) - log(cs));
                if (!isfinite(gn)) s_bad = 1;
                d.g[pin ^ 1][tid] = gn;
            }
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
                    // polish only when the FP32 sweeps stalled short of tol; a
                    // residual that met a tol above the FP32 noise threshold
                    // goes straight to the exact check
                    const bool met = ctl->r_last < ctl->tol_fast && ctl->tol >= P.stall_below;
                    if (phase == kPhFast && P.polish_iters > 0 && ctl->iter < ctl->max_iter && !met) {
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
                int np = parts;
                if (ctl->iter >= kFineIter && d.rpp > kFineRows) {
                    np = (int)((d.I + kFineRows - 1) / kFineRows);
                    tab[k].rpp = kFineRows;
                    tab[k].parts = np;
                }
                s_parts = np;
                const int par = (next == 2 ? ctl->check_iter : ctl->iter) & 1;
                s_flags = (ctl->has_prev ? kItPrev : 0) | (par ? kItPar : 0) | (next == 2 ? kItCheck : 0);
                s_base = atomicAdd(&out.cnt[next == 0 ? 0 : 1], np);
                out.inst[atomicAdd(&out.cnt[2], 1)] = k;
            }
        }
        __syncthreads();
        if (s_list >= 0) {
            BItem* dst = (s_list == 0 ? out.it32 : out.it64) + s_base;
            for (int p = tid; p < s_parts; p += 1024) dst[p] = BItem{k, p, s_flags, 0};
        }
        __syncthreads();  // shared state is rewritten by the next instance
    }
}

// Everything one admitted instance needs on the device, staged by the host
// in one block for the whole admission.
struct AdmJob {
    BInst d;
    Ctl ci;
    SolveParams sp;
    SolveParams* prm_dst;
    const double* a_src;  // marginals to copy into d.a / d.b
    const double* b_src;
    const double* f0;  // warm start (with g0) or null
    const double* g0;
    int slot;
    int item_base;  // offset of its items among this admission's items
    int inst_pos;   // position among this admission's instances
    int pad_;
};

// One workgroup per admitted instance: copies and checks its marginals
// (a_i > 0 and b_j > 0 finite, |sum a - sum b| <= 1e-12 sum a), sets up its
// starting potentials, writes its table entry, control block (mass = sum a;
// an instance that fails the checks is marked done with numeric_bad = 2
// before any work runs) and constants, and appends its first sweep items to a
// list generation that no kernel is using. The list counters move afterwards
// (k_bcount), so every workgroup reads the same base.
__global__ __launch_bounds__(256) void k_badmit_jobs(const AdmJob* __restrict__ jobs, BInst* tab, Ctl* ctls,
                                                     BList l) {
    const AdmJob& J = jobs[blockIdx.x];
    const BInst& d = J.d;
    double* a = const_cast<double*>(d.a);
    double* b = const_cast<double*>(d.b);
    __shared__ double red[4][2];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    int flag = 0;
    for (int64_t i = threadIdx.x; i < d.I; i += blockDim.x) {
        const double v = J.a_src[i];
        a[i] = v;
        flag |= !(v > 0.0 && isfinite(v));
        sa += v;
        if (J.f0) d.f[0][i] = J.f0[i];
    }
    for (int j = threadIdx.x; j < d.J; j += blockDim.x) {
        const double v = J.b_src[j];
        b[j] = v;
        flag |= !(v > 0.0 && isfinite(v));
        sb += v;
        d.g[0][j] = J.g0 ? J.g0[j] : 0.0;
    }
    if (flag) bad = 1;
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[w][0] = sa;
        red[w][1] = sb;
    }
    const int base = l.cnt[0] + J.item_base;
    const int flags = J.f0 ? kItPrev : 0;
    for (int p = threadIdx.x; p < d.parts; p += blockDim.x) l.it32[base + p] = BItem{J.slot, p, flags, 0};
    __syncthreads();
    if (threadIdx.x == 0) {
        const double ta = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        const double tb = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
        Ctl c = J.ci;
        c.mass = ta;
        if (bad || !(fabs(ta - tb) <= 1e-12 * ta)) {
            c.numeric_bad = 2;
            c.done = 1;
            c.phase = kPhDone;
            c.result_iter = 0;
            c.chk_violation = __builtin_nan("");
        }
        ctls[J.slot] = c;
        tab[J.slot] = d;
        *J.prm_dst = J.sp;
        l.inst[l.cnt[2] + J.inst_pos] = J.slot;
    }
}

// Advances the counters of a list generation after appends.
__global__ void k_bcount(BList l, int n_items, int n_insts) {
    if (threadIdx.x == 0) {
        l.cnt[0] += n_items;
        l.cnt[2] += n_insts;
    }
}

// Re-partitions instances that have not started (rows per part rpp) and
// queues their first sweep items in an emptied list generation.
__global__ __launch_bounds__(256) void k_brelayout(BInst* tab, const int* __restrict__ slots,
                                                   const int* __restrict__ bases, int64_t rpp, BList l) {
    const int k = slots[blockIdx.x];
    const int64_t I = tab[k].I;
    const int parts = (int)((I + rpp - 1) / rpp);
    const int flags = tab[k].ctl->has_prev ? kItPrev : 0;
    for (int p = threadIdx.x; p < parts; p += blockDim.x) l.it32[bases[blockIdx.x] + p] = BItem{k, p, flags, 0};
    __syncthreads();
    if (threadIdx.x == 0) {
        tab[k].rpp = rpp;
        tab[k].parts = parts;
        l.inst[blockIdx.x] = k;
    }
}

// Clears a list generation (all three counters).
__global__ void k_bclear(BList l) {
    if (threadIdx.x < 3) l.cnt[threadIdx.x] = 0;
}

// Batched padded copies of cost sources (one job per blockIdx.y):
// dst[i ld + j] = cost(i, j) for j < J, +inf for J <= j < ld. kind 0: dense C;
// 1: rates, c = inv_scale / R.
struct PadJob {
    const void* src;
    float* dst;
    int64_t I, lds, ld;
    double inv_scale;
    int J;
    int kind;
    int f64;
    int pad_;
};

// One wavefront per row (4 per workgroup, rows grid-strided over
// gridDim.x workgroups per job): lane l writes the 16-byte groups l, l + 64,
// ... of the padded row (ld / 4 <= 128 of them), reading its four source
// elements one by one (the source stride need not be a multiple of 4).
constexpr int kPadRowsPerBlock = 4;
__global__ __launch_bounds__(256) void k_bpad_jobs(const PadJob* __restrict__ jobs) {
    const PadJob& P = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int nq = (int)(P.ld / 4);
    const float* s32 = (const float*)P.src;
    const double* s64 = (const double*)P.src;
    for (int64_t i = (int64_t)blockIdx.x * kPadRowsPerBlock + (threadIdx.x >> 6); i < P.I;
         i += (int64_t)gridDim.x * kPadRowsPerBlock) {
        float4* drow = reinterpret_cast<float4*>(P.dst + i * P.ld);
        const int64_t e0 = i * P.lds;
        for (int q = lane; q < nq; q += 64) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 4 * q + u;
                float x = __builtin_huge_valf();
                if (j < P.J) {
                    const double c = P.f64 ? s64[e0 + j] : (double)s32[e0 + j];
                    x = P.kind == 0 ? (float)c : (float)((1.0 / c) * P.inv_scale);
                }
                v[u] = x;
            }
            drow[q] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// Costs regenerated from positions, set up for a whole admission group in
// two launches. Job k covers the flat block range [blk0, blk0 + nblk) of each
// launch (prepass: 4 rows per block, geometry only; materialisation: 8 rows
// per block); a block finds its job by a binary search of the job starts
// (the last job whose range starts at or before the block).
struct GeoJob {
    GeoSrc geo;        // geometry (kind 0): positions, set-up sums, constants
    EuclidSrc dist;    // distances (kind 1)
    double* s_all;     // geometry set-up outputs (the arrays geo reads)
    double* s_ex;
    int* j1;
    float* dst;        // I x ld padded FP32 cost
    int64_t I, ld;
    int J;
    int kind;
    int pre_blk0, pre_nblk;  // prepass blocks (0 for distances)
    int mat_blk0, mat_nblk;  // materialisation blocks
};

constexpr int kGeoJobRowsPre = 4;  // 256 threads, a wavefront per row
constexpr int kGeoJobRowsMat = 8;  // 512 threads, a wavefront per row

__device__ __forceinline__ int find_job(const GeoJob* jobs, int n, int b, bool pre) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((pre ? jobs[mid].pre_blk0 : jobs[mid].mat_blk0) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_bgeo_prepass_jobs(const GeoJob* __restrict__ jobs, int n) {
    __shared__ float2 xy[kBatchMaxJ];
    const int k = find_job(jobs, n, blockIdx.x, true);
    const GeoJob& G = jobs[k];
    const int rb = (int)blockIdx.x - G.pre_blk0;
    if (G.kind != 0 || rb < 0 || rb >= G.pre_nblk) return;
    for (int c = threadIdx.x; c < G.J; c += blockDim.x) xy[c] = reinterpret_cast<const float2*>(G.geo.rrh_xy)[c];
    __syncthreads();
    const int64_t i = (int64_t)rb * kGeoJobRowsPre + threadIdx.x / 64;
    if (i >= G.I) return;
    geo_prepass_row<kBatchMaxJ / 64>(G.geo, i, G.J, xy, threadIdx.x & 63, G.s_all, G.s_ex, G.j1);
}

__global__ __launch_bounds__(512) void k_bmat_jobs(const GeoJob* __restrict__ jobs, int n) {
    __shared__ double sm[kBatchMaxJ + 1];
    const int k = find_job(jobs, n, blockIdx.x, false);
    const GeoJob& G = jobs[k];
    const int rb = (int)blockIdx.x - G.mat_blk0;
    if (rb < 0 || rb >= G.mat_nblk) return;
    if (G.kind == 0) G.geo.stage(sm, G.J);
    else G.dist.stage(sm, G.J);
    __syncthreads();
    const int64_t i = (int64_t)rb * kGeoJobRowsMat + threadIdx.x / 64;
    if (i >= G.I) return;
    if (G.kind == 0) materialize_row(G.geo, i, G.J, G.ld, G.dst, sm, threadIdx.x & 63);
    else materialize_row(G.dist, i, G.J, G.ld, G.dst, sm, threadIdx.x & 63);
}

}  // namespace otk
