// Kernels of the snapshot solve: B traffic snapshots (device marginals a_s,
// one per snapshot) over one cost matrix C and one RRH marginal b, solved
// together in the scaling form of the Sinkhorn iteration (Sec. III-B),
//   u_s = a_s / (K v_s),   v_s = b / (K^T u_s),   pi_s = diag(u_s) K diag(v_s),
// with the kernel stabilised by the potentials (fbar, gbar) of a reference
// solve: K_ij = exp((fbar_i + gbar_j - C_ij) / eps), so that u and v stay near
// 1 and the potentials of snapshot s are fbar + eps ln u_s, gbar + eps ln v_s.
// Stacking the snapshots as columns turns both half-steps into GEMMs with a
// K-dimension of J and I respectively:
//   P = K V   (I x J) . (J x B)        Q = K^T U   (J x I) . (I x B)
// run on the matrix cores (v_mfma_f32_16x16x32_bf16). K (and its transpose,
// so both GEMMs read their A operand along contiguous memory), U and V are
// each split into BF16 high and low parts (x = hi + lo: about 16 significant
// bits instead of BF16's 8, so that a plan concentrated on few RRHs per
// device does not inherit the 2^-9 relative rounding of a single BF16 K
// entry as its marginal error). A product is Kh Xh + Kh Xl + Kl Xh (the
// Kl Xl term is below FP32 accumulation), every product accumulating in FP32.
//
// MFMA 16x16x32 lane layout (lane l of the 64-lane wavefront):
//   A (16 x 32): row l % 16, k = 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16): col l % 16, k = 8 (l / 16) .. 8 (l / 16) + 7
//   D (16 x 16): col l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3
#pragma once

#include "kernels.h"

namespace otk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSnapB = 64;     // snapshots per GEMM (4 column tiles of 16)
constexpr int kSnapNT = kSnapB / 16;

// Round-to-nearest-even FP32 -> BF16 (bit pattern); infinities pass, NaNs
// stay NaN (quiet bit set when the payload would round away). Written as a
// select so that a wave does not branch on it.
__device__ __forceinline__ unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    const unsigned special = (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    const unsigned rne = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    return (unsigned short)((u & 0x7f800000u) == 0x7f800000u ? special : rne);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Device state of a snapshot solve.
struct SnapArgs {
    int64_t I, Ip;   // rows; rows padded to a multiple of 32 (K-dimension of Q)
    int J, Jp;       // columns; padded to a multiple of 32 (K-dimension of P)
    int B;           // live snapshots (<= kSnapB)
    int splits;      // K-splits of the column GEMM
    int64_t rows_per_split;  // multiple of 32
    const unsigned short* K;   // Ip x Jp BF16 high part, zero padded
    const unsigned short* Kt;  // Jp x Ip BF16 high part, zero padded
    const unsigned short* Kl;  // Ip x Jp BF16 low part
    const unsigned short* Ktl; // Jp x Ip BF16 low part
    const double* A;           // kSnapB x I marginals a_s (rows >= B unused)
    const double* b;           // J
    float* U;                  // kSnapB x Ip
    unsigned short* Uh;        // kSnapB x Ip, BF16 high part of U
    unsigned short* Ul;        // kSnapB x Ip, BF16 low part
    float* V;                  // kSnapB x Jp
    unsigned short* Vh;        // kSnapB x Jp
    unsigned short* Vl;        // kSnapB x Jp
    float* Qpart;              // splits x kSnapB x Jp
    double* res;               // kSnapB x kResParts: column residual of the last combined iterate
    double* mass;              // kSnapB: sum a_s
    int* ctl;                  // [0] iterations done, [1] stop, [2] max_iter, [3] result iteration
    double tol;
};

// Splits x (FP32) into BF16 high and low parts.
__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

// Builds the stabilised kernel as BF16 high / low parts and their
// transposes, through 32 x 32 LDS tiles: K_ij = exp2((fbar_i + gbar_j - C_ij)
// log2(e) / eps) rounded to FP32, zero outside I x J.
__global__ __launch_bounds__(256) void k_snap_build(const float* C, int64_t ldc, int64_t I, int J, int64_t Ip, int Jp,
                                                    const double* fbar, const double* gbar, double kk,
                                                    unsigned short* K, unsigned short* Kt, unsigned short* Kl,
                                                    unsigned short* Ktl) {
    __shared__ unsigned short th[32][33], tl[32][33];
    const int64_t i0 = (int64_t)blockIdx.y * 32;
    const int j0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r;
        const int j = j0 + tx;
        float v = 0.0f;
        if (i < I && j < J) v = (float)exp2((fbar[i] + gbar[j] - (double)C[i * ldc + j]) * kk);
        unsigned short h, l;
        split_bf16(v, h, l);
        K[i * Jp + j] = h;
        Kl[i * Jp + j] = l;
        th[r][tx] = h;
        tl[r][tx] = l;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t o = (int64_t)(j0 + r) * Ip + i0 + tx;
        Kt[o] = th[tx][r];
        Ktl[o] = tl[tx][r];
    }
}

// Sets the scaling vectors of a cold start: v = 1 on live (s, j), 0 elsewhere.
__global__ void k_snap_init(SnapArgs S) {
    const int64_t n = (int64_t)kSnapB * S.Jp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / S.Jp), j = (int)(e - (int64_t)s * S.Jp);
        const float v = (s < S.B && j < S.J) ? 1.0f : 0.0f;
        unsigned short hi, lo;
        split_bf16(v, hi, lo);
        S.V[e] = v;
        S.Vh[e] = hi;
        S.Vl[e] = lo;
    }
    if (blockIdx.x == 0)
        for (int q = threadIdx.x; q < kSnapB * 4; q += blockDim.x) S.res[q] = __builtin_huge_val();
}

__device__ __forceinline__ bf16x8 load8(const unsigned short* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}

// Stop decision, taken identically by every wave of the row pass from the
// residuals of the last combine (kResParts column quarters per snapshot,
// summed in a fixed order): all live snapshots met tol, or the iteration cap.
// Lane s takes snapshot s (kSnapB is the wavefront width) and the wave takes
// the maximum; a NaN residual counts as 0, as in a sequential fmax from 0.
// Every lane of the wave must be active.
constexpr int kResParts = 4;
static_assert(kSnapB == 64, "one snapshot per lane of the stop decision");
__device__ __forceinline__ double snap_residual(const SnapArgs& S, int s) {
    const double* r = S.res + (int64_t)s * kResParts;
    return ((r[0] + r[1]) + (r[2] + r[3])) / S.mass[s];
}
__device__ __forceinline__ bool snap_stop(const SnapArgs& S, int lane) {
    if (S.ctl[1]) return true;
    const double r = wave_max(lane < S.B ? fmax(0.0, snap_residual(S, lane)) : 0.0);
    return (r < S.tol) || (S.ctl[0] >= S.ctl[2]);
}

// One wave's share of RT stacked 16 x kSnapB output tiles: K-steps k0 = kbeg,
// kbeg + kstride, ... < kend of A = Ah + Al (RT tiles of 16 rows, tile r's
// lane row at ahrow / alrow + r astride) times the hi and lo parts of B^T
// (kSnapB rows, row stride ldb). Each B fragment serves all RT tiles. The
// steps go in groups of G whose fragments are all loaded before the group's
// first product, so that a wave with at most G steps waits for memory once;
// a step of a group past kend reads the last step's (in-bounds) fragments
// and multiplies a zeroed A fragment. kbeg, kend and kstride are multiples
// of 32.
template <int RT, int G>
__device__ __forceinline__ void snap_tile(const unsigned short* ahrow, const unsigned short* alrow, int64_t astride,
                                          const unsigned short* bh, const unsigned short* bl, int64_t ldb,
                                          int64_t kbeg, int64_t kend, int64_t kstride, int lane,
                                          f32x4 (&acc)[RT][kSnapNT]) {
    const int m = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < kSnapNT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (kbeg >= kend) return;
    const bf16x8 zero = {};
    for (int64_t kb = kbeg; kb < kend; kb += G * kstride) {
        bf16x8 a[G][RT], al[G][RT], h[G][kSnapNT], l[G][kSnapNT];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t k0 = kb + g * kstride;
            const int64_t kc = k0 < kend ? k0 : kend - 32;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                a[g][r] = load8(ahrow + r * astride + kc + kq);
                al[g][r] = load8(alrow + r * astride + kc + kq);
            }
#pragma unroll
            for (int t = 0; t < kSnapNT; ++t) {
                const int64_t o = (int64_t)(t * 16 + m) * ldb + kc + kq;
                h[g][t] = load8(bh + o);
                l[g][t] = load8(bl + o);
            }
        }
        // keep the scheduler from sinking the group's loads between its
        // products (it would, to save registers)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const bool live = kb + g * kstride < kend;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const bf16x8 ca = live ? a[g][r] : zero, cal = live ? al[g][r] : zero;
#pragma unroll
                for (int t = 0; t < kSnapNT; ++t) {
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, h[g][t], acc[r][t], 0, 0, 0);
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ca, l[g][t], acc[r][t], 0, 0, 0);
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cal, h[g][t], acc[r][t], 0, 0, 0);
                }
            }
        }
    }
}

// Sums the four waves' partial tiles through LDS in wave order, for RT
// tiles; wave w < RT returns with the total of tile w.
template <int RT>
__device__ __forceinline__ void snap_reduce4(f32x4 (&acc)[RT][kSnapNT], int w, int lane, f32x4 (&tot)[kSnapNT]) {
    static_assert(RT <= 4, "one reducing wave per tile");
    __shared__ f32x4 red[4][RT][kSnapNT][64];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < kSnapNT; ++t) red[w][r][t][lane] = acc[r][t];
    __syncthreads();
    if (w < RT)
#pragma unroll
        for (int t = 0; t < kSnapNT; ++t)
            tot[t] = ((red[0][w][t][lane] + red[1][w][t][lane]) + red[2][w][t][lane]) + red[3][w][t][lane];
}

// Row tiles of 16 per wave in the row GEMM, column tiles of 16 per wave in
// the column GEMM.
constexpr int kSnapRowRT = 2;
constexpr int kSnapColRT = 2;
// K-steps loaded together per wave: 1 measured fastest at 64 snapshots x
// 20000 x 400 (groups of 2 and 4 lower the occupancy more than they save)
constexpr int kSnapGroup = 1;

// Row half-step: P = K V for 16 kSnapRowRT rows per workgroup (the four waves
// take every fourth K-step and are summed in LDS), then u = a / P (0 on
// padded rows and snapshots), stored as FP32 and as BF16 hi / lo.
__global__ __launch_bounds__(256) void k_snap_rows(SnapArgs S) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (snap_stop(S, lane)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && !S.ctl[1]) {
            S.ctl[1] = 1;
            S.ctl[3] = S.ctl[0];
        }
        return;
    }
    const int64_t i0 = (int64_t)blockIdx.x * (16 * kSnapRowRT);
    const int m = lane & 15;
    // D: column = snapshot t * 16 + m, rows i0 + 16 w + 4 (lane / 16) + q.
    // The marginals this wave divides by are loaded first (entry 0 for padded
    // rows and snapshots, whose u is 0), so that they arrive with the GEMM's
    // fragments rather than one by one after it.
    const int64_t ib = i0 + 16 * (w % kSnapRowRT) + (lane >> 4) * 4;
    double av[kSnapNT][4];
#pragma unroll
    for (int t = 0; t < kSnapNT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = t * 16 + m;
            const int64_t i = ib + q;
            av[t][q] = S.A[(s < S.B && i < S.I) ? (int64_t)s * S.I + i : 0];
        }
    f32x4 acc[kSnapRowRT][kSnapNT], tot[kSnapNT];
    snap_tile<kSnapRowRT, kSnapGroup>(S.K + (i0 + m) * S.Jp, S.Kl + (i0 + m) * S.Jp, 16 * S.Jp, S.Vh, S.Vl, S.Jp,
                                      (int64_t)w * 32, S.Jp, 128, lane, acc);
    snap_reduce4<kSnapRowRT>(acc, w, lane, tot);
    if (w >= kSnapRowRT) return;
#pragma unroll
    for (int t = 0; t < kSnapNT; ++t) {
        const int s = t * 16 + m;
        float u[4];
        unsigned short hi[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x = (float)(av[t][q] / (double)tot[t][q]);
            u[q] = (s < S.B && ib + q < S.I) ? x : 0.0f;
            split_bf16(u[q], hi[q], lo[q]);
        }
        const int64_t o = (int64_t)s * S.Ip + ib;
        *reinterpret_cast<float4*>(S.U + o) = make_float4(u[0], u[1], u[2], u[3]);
        *reinterpret_cast<ushort4*>(S.Uh + o) = make_ushort4(hi[0], hi[1], hi[2], hi[3]);
        *reinterpret_cast<ushort4*>(S.Ul + o) = make_ushort4(lo[0], lo[1], lo[2], lo[3]);
    }
}

// Column half-step, split along i: Qpart[split] = K^T[j-tiles, rows of
// split] U for 16 kSnapColRT columns per workgroup (the four waves take
// every fourth K-step and are summed in LDS).
__global__ __launch_bounds__(256) void k_snap_cols(SnapArgs S) {
    if (S.ctl[1]) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j0 = blockIdx.x * (16 * kSnapColRT), split = blockIdx.y;
    const int m = lane & 15;
    const int64_t r0 = (int64_t)split * S.rows_per_split;
    const int64_t r1 = min(S.Ip, r0 + S.rows_per_split);
    f32x4 acc[kSnapColRT][kSnapNT], tot[kSnapNT];
    snap_tile<kSnapColRT, kSnapGroup>(S.Kt + (int64_t)(j0 + m) * S.Ip, S.Ktl + (int64_t)(j0 + m) * S.Ip, 16 * S.Ip, S.Uh, S.Ul,
                          S.Ip, r0 + (int64_t)w * 32, r1, 128, lane, acc);
    snap_reduce4<kSnapColRT>(acc, w, lane, tot);
    if (w >= kSnapColRT) return;
    const int jb = j0 + 16 * w + (lane >> 4) * 4;
#pragma unroll
    for (int t = 0; t < kSnapNT; ++t) {
        const int s = t * 16 + m;
        float* o = S.Qpart + ((int64_t)split * kSnapB + s) * S.Jp + jb;
        *reinterpret_cast<float4*>(o) = make_float4(tot[t][0], tot[t][1], tot[t][2], tot[t][3]);
    }
}

// Column combine, workgroup (s, quarter): for its quarter of the columns,
// Q = sum of the splits (fixed order, FP64), the column residual of the
// iterate (u, v_old) and v = b / Q.
__global__ __launch_bounds__(256) void k_snap_combine(SnapArgs S) {
    if (S.ctl[1]) return;
    const int s = blockIdx.x, quarter = blockIdx.y;
    const int jq = (S.Jp / 4 + 63) / 64 * 64;  // columns per quarter
    __shared__ double red[4];
    double r = 0.0;
    const int jend = min(S.Jp, (quarter + 1) * jq);
    for (int j = quarter * jq + threadIdx.x; j < jend; j += blockDim.x) {
        const int64_t e = (int64_t)s * S.Jp + j;
        float v = 0.0f;
        if (s < S.B && j < S.J) {
            const float* qp = S.Qpart + (int64_t)s * S.Jp + j;
            const int64_t step = (int64_t)kSnapB * S.Jp;
            double q = 0.0;
            int p = 0;
            for (; p + 8 <= S.splits; p += 8) {
                float x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = qp[(p + u) * step];
#pragma unroll
                for (int u = 0; u < 8; ++u) q += (double)x[u];
            }
            for (; p < S.splits; ++p) q += (double)qp[p * step];
            r += fabs((double)S.V[e] * q - S.b[j]);
            v = (float)(S.b[j] / q);
        }
        unsigned short hi, lo;
        split_bf16(v, hi, lo);
        S.V[e] = v;
        S.Vh[e] = hi;
        S.Vl[e] = lo;
    }
    r = wave_sum(r);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        S.res[(int64_t)s * kResParts + quarter] = (red[0] + red[1]) + (red[2] + red[3]);
        if (s == 0 && quarter == 0) S.ctl[0] += 1;
    }
}

// Snapshot marginals on the device: abar_i = mean over s of A[s][i], and a
// flag when any entry is not positive and finite.
__global__ void k_snap_mean(const double* A, int B, int64_t I, double* abar, int* bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I; i += (int64_t)gridDim.x * blockDim.x) {
        double t = 0.0;
        int f = 0;
        for (int s = 0; s < B; ++s) {
            const double v = A[(int64_t)s * I + i];
            f |= !(v > 0.0 && isfinite(v));
            t += v;
        }
        abar[i] = t / B;
        if (f) *bad = 1;
    }
}

// mass[s] = sum_i A[s][i] (fixed order), one workgroup per snapshot; 1 for
// padded snapshots.
__global__ __launch_bounds__(256) void k_snap_mass(const double* A, int B, int64_t I, double* mass) {
    const int s = blockIdx.x;
    __shared__ double red[4];
    double t = 0.0;
    if (s < B)
        for (int64_t i = threadIdx.x; i < I; i += blockDim.x) t += A[(int64_t)s * I + i];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) mass[s] = s < B ? (red[0] + red[1]) + (red[2] + red[3]) : 1.0;
}

// Potentials of every live snapshot: F[s] = fbar + eps ln u_s (I),
// G[s] = gbar + eps ln v_s (J), FP64.
__global__ void k_snap_all_potentials(SnapArgs S, const double* fbar, const double* gbar, double eps, double* F,
                                      double* G) {
    const int s = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.I; i += (int64_t)gridDim.x * blockDim.x)
        F[(int64_t)s * S.I + i] = fbar[i] + eps * log((double)S.U[(int64_t)s * S.Ip + i]);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < S.J; j += (int64_t)gridDim.x * blockDim.x)
        G[(int64_t)s * S.J + j] = gbar[j] + eps * log((double)S.V[(int64_t)s * S.Jp + j]);
}

// Exact FP64 check of every snapshot in one launch: workgroup (chunk, s)
// takes rows [chunk rpc, (chunk + 1) rpc) of snapshot s and writes its column
// partials and five row statistics (check_rows).
template <int NCH>
__global__ __launch_bounds__(512) void k_snap_check(const float* C, int64_t ldc, int64_t I, int J, int64_t rpc,
                                                    const double* A, const double* F, const double* G, double kk,
                                                    double* col_part, double* stat_part) {
    const int s = blockIdx.y, chunk = blockIdx.x, nchunk = gridDim.x;
    CheckJob cj;
    cj.r0 = (int64_t)chunk * rpc;
    cj.r1 = min(I, cj.r0 + rpc);
    cj.J = J;
    cj.nch = (J + 63) / 64;
    cj.kk = kk;
    cj.a = A + (int64_t)s * I;
    cj.f = F + (int64_t)s * I;
    cj.g = G + (int64_t)s * J;
    cj.col_out = col_part + ((int64_t)s * nchunk + chunk) * J;
    cj.stat_out = stat_part + ((int64_t)s * nchunk + chunk) * 5;
    check_rows<DenseSrc<float>, 1, NCH, 8>(cj, DenseSrc<float>{C, ldc});
}

// Per snapshot: column sums of the check, the statistics, into out[s * 8]:
// violation, <C, pi>, reg. objective, dual, mass, row residual, col residual.
__global__ __launch_bounds__(256) void k_snap_check_finish(int nchunk, int J, const double* b, const double* G,
                                                           const double* col_part, const double* stat_part,
                                                           const double* mass, double eps, double* out) {
    const int s = blockIdx.x;
    __shared__ double red[4][7];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
        double cs = 0.0;
        for (int c = 0; c < nchunk; ++c) cs += col_part[((int64_t)s * nchunk + c) * J + j];
        v[5] += fabs(cs - b[j]);
        v[6] += G[(int64_t)s * J + j] * b[j];
    }
    for (int c = threadIdx.x; c < nchunk; c += blockDim.x)
        for (int u = 0; u < 5; ++u) v[u] += stat_part[((int64_t)s * nchunk + c) * 5 + u];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int u = 0; u < 7; ++u) {
        const double t = wave_sum(v[u]);
        if (lane == 0) red[w][u] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[7];
        for (int u = 0; u < 7; ++u) t[u] = (red[0][u] + red[1][u]) + (red[2][u] + red[3][u]);
        double* o = out + (int64_t)s * 8;
        o[0] = (t[0] + t[5]) / mass[s];
        o[1] = t[1];
        o[2] = t[1] + eps * t[2];
        o[3] = t[4] + t[6] - eps * t[3];
        o[4] = t[3];
        o[5] = t[0];
        o[6] = t[5];
    }
}

}  // namespace otk
