// Association quality and the maxSINR rule (Sec. II-B, Sec. IV):
//
//  k_loads      per-RRH load of the transport plan x = exp((f + g - C)/eps),
//               sum_i C_ij x_ij, or (second pass, with rho known) each
//               device's completion-time sum sum_j C_ij x_ij / (1 - rho_j),
//               from the FP64 cost functor; one row per wavefront step, lane
//               = column, FP64 throughout; workgroup partials per column.
//  k_cols_fin   fixed-order sums of the workgroup partials: rho_j = kappa
//               load_j and E[N_j] = rho_j / (1 - rho_j) (processor sharing);
//  k_rows_fin   the total of the device completion times (time pass).
//  k_maxsinr    the maxSINR rule: each device to its cheapest RRH (highest
//               rate, lowest index on ties) and, per workgroup, the traffic
//               a_i it sends to every RRH, summed in row order;
//  k_cols_fin   fixed-order column sums of such partials (Lambda_j).
#pragma once

#include "kernels.h"

namespace otk {

struct LoadArgs {
    int64_t I;
    int J;
    int nch;  // column chunks of 64 * VEC
    int64_t rows_per_block;
    double kk;        // log2(e) / eps
    const double* a;  // row sums (time pass)
    const double* f;
    const double* g;
    const double* rho;  // null: load pass; else time pass with these loads
    double* col_part;   // load pass: gridDim.x x J partial loads
    double* row_part;   // time pass: gridDim.x x 2 (sum of T_i / tau, devices on overloaded RRHs)
};

template <class Src, int VEC, int NCH, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_loads(LoadArgs A, Src src) {
    extern __shared__ double sm[];
    const double kk = A.kk;
    const int J = A.J, nch = A.nch;
    const int ncols = nch * kWave * VEC;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t r0 = (int64_t)blockIdx.x * A.rows_per_block;
    const int64_t r1 = min(A.I, r0 + A.rows_per_block);
    const bool time_pass = A.rho != nullptr;
    src.stage(sm, J);
    double gsr[NCH][VEC], inv1[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int col = (ch * kWave + lane) * VEC + v;
            const bool ok = ch < nch && col < J;
            gsr[ch][v] = ok ? A.g[col] * kk : -pinf64();
            // 1 / (1 - rho_j); an overloaded RRH (rho_j >= 1) is marked by -1
            inv1[ch][v] = (ok && time_pass) ? (A.rho[col] < 1.0 ? 1.0 / (1.0 - A.rho[col]) : -1.0) : 0.0;
        }
    __syncthreads();
    double acc[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[ch][v] = 0.0;
    double tsum = 0.0, nover = 0.0;  // (lane 0 of each wave)
    for (int64_t i = r0 + w; i < r1; i += WAVES) {
        auto row = src.row(i);
        const double fk = A.f[i] * kk;
        double ts = 0.0;
        bool over = false;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            if (ch < nch) {
                const int col0 = (ch * kWave + lane) * VEC;
                double c[VEC];
                src.template get<true, VEC>(row, i, col0, J, sm, c);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    if (col0 + v < J) {
                        const double p = exp2(fk + fma(c[v], -kk, gsr[ch][v]));
                        const double cp = c[v] * p;
                        if (time_pass) {
                            if (inv1[ch][v] < 0.0) over |= p > 0.0;
                            else ts = fma(cp, inv1[ch][v], ts);
                        } else {
                            acc[ch][v] += cp;
                        }
                    }
                }
            }
        }
        if (time_pass) {
            ts = wave_sum(ts);
            const bool ov = __any(over);
            if (lane == 0) {
                if (ov) nover += 1.0;
                else tsum += ts / A.a[i];
            }
        }
    }
    if (time_pass) {
        __shared__ double wt[WAVES][2];
        if (lane == 0) { wt[w][0] = tsum; wt[w][1] = nover; }
        __syncthreads();
        if (threadIdx.x < 2) {
            double s = 0.0;
            for (int q = 0; q < WAVES; ++q) s += wt[q][threadIdx.x];
            A.row_part[(int64_t)blockIdx.x * 2 + threadIdx.x] = s;
        }
        return;
    }
    __syncthreads();
    block_tree<NCH, VEC, WAVES>(acc, nch, sm, ncols, w, lane);
    if (w == 0) {
        double* out = A.col_part + (int64_t)blockIdx.x * J;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (ch < nch)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const int col = (ch * kWave + lane) * VEC + v;
                    if (col < J) out[col] = acc[ch][v];
                }
    }
}

// Column sums of `nb` workgroup partials: out[j] = scale * sum_b part[b][j];
// with en set, en[j] = out[j] / (1 - out[j]) for out[j] < 1, else +inf.
// kFinCols columns per workgroup of 1024 threads; the 64 threads of a column
// each add every 64th partial (eight loads in flight), then one thread adds
// their 64 sums in order: a fixed order, with a thousand partials in flight
// per column instead of one after another.
constexpr int kFinCols = 16;
static __global__ __launch_bounds__(1024) void k_cols_fin(const double* part, int nb, int J, double scale, double* out,
                                                          double* en) {
    static_assert(kFinCols * 64 == 1024, "64 threads per column");
    const int c = threadIdx.x % kFinCols, r = threadIdx.x / kFinCols;
    const int j = blockIdx.x * kFinCols + c;
    double s = 0.0;
    if (j < J) {
        int q = r;
        for (; q + 7 * 64 < nb; q += 8 * 64) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(q + u * 64) * J + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; q < nb; q += 64) s += part[(int64_t)q * J + j];
    }
    __shared__ double red[64][kFinCols + 1];
    red[r][c] = s;
    __syncthreads();
    const int jj = blockIdx.x * kFinCols + (int)threadIdx.x;
    if (threadIdx.x < kFinCols && jj < J) {
        double t = 0.0;
        for (int q = 0; q < 64; ++q) t += red[q][threadIdx.x];
        t *= scale;
        out[jj] = t;
        if (en) en[jj] = t < 1.0 ? t / (1.0 - t) : pinf64();
    }
}

// Sum of the time pass's workgroup pairs: out[0] = sum T_i / tau, out[1] =
// devices using an overloaded RRH. One workgroup of 256 threads: thread t
// adds pairs t, t + 256, ..., then thread 0 adds the 256 sums in order.
static __global__ __launch_bounds__(256) void k_rows_fin(const double* row_part, int nb, double* out) {
    __shared__ double red[256][2];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        s0 += row_part[(int64_t)b * 2];
        s1 += row_part[(int64_t)b * 2 + 1];
    }
    red[threadIdx.x][0] = s0;
    red[threadIdx.x][1] = s1;
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
        for (int q = 0; q < 256; ++q) t += red[q][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// maxSINR rule. A workgroup of 256 threads owns rows [b rpb, (b + 1) rpb) and
// walks them in chunks of kMaxsinrRows: one wavefront per row finds the
// cheapest RRH (FP64 cost functor, lowest index on ties); then thread t adds,
// for its columns j = t, t + 256, ..., the traffic a_i of the chunk's rows
// that chose j, in row order.
constexpr int kMaxsinrRows = 64;
constexpr int kMaxsinrCols = 8;  // columns per thread: J <= 2048

template <class Src>
__global__ __launch_bounds__(256) void k_maxsinr(int64_t I, int J, int64_t rpb, const double* a, Src src,
                                                 int32_t* assoc, double* col_part) {
    extern __shared__ double sm[];
    __shared__ int s_j[kMaxsinrRows];
    __shared__ double s_a[kMaxsinrRows];
    src.stage(sm, J);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = min(I, r0 + rpb);
    double acc[kMaxsinrCols];
#pragma unroll
    for (int u = 0; u < kMaxsinrCols; ++u) acc[u] = 0.0;
    for (int64_t c0 = r0; c0 < r1; c0 += kMaxsinrRows) {
        for (int lr = w; lr < kMaxsinrRows; lr += 4) {
            const int64_t i = c0 + lr;
            if (i >= r1) {
                if (lane == 0) { s_j[lr] = -1; s_a[lr] = 0.0; }
                continue;
            }
            auto row = src.row(i);
            double best = pinf64();
            int bj = 0x7fffffff;
            for (int j = lane; j < J; j += 64) {
                const double c = src.at64(row, i, j, sm);
                if (c < best || (c == best && j < bj)) { best = c; bj = j; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oj = __shfl_xor(bj, o, 64);
                if (ob < best || (ob == best && oj < bj)) { best = ob; bj = oj; }
            }
            if (lane == 0) {
                if (bj >= J) bj = 0;  // (every cost +inf: the first RRH)
                s_j[lr] = bj;
                s_a[lr] = a[i];
                if (assoc) assoc[i] = bj;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxsinrCols; ++u) {
            const int j = (int)threadIdx.x + 256 * u;
            if (j < J)
                for (int lr = 0; lr < kMaxsinrRows; ++lr)
                    if (s_j[lr] == j) acc[u] += s_a[lr];
        }
        __syncthreads();  // the chunk's LDS is rewritten next
    }
#pragma unroll
    for (int u = 0; u < kMaxsinrCols; ++u) {
        const int j = (int)threadIdx.x + 256 * u;
        if (j < J) col_part[(int64_t)blockIdx.x * J + j] = acc[u];
    }
}

}  // namespace otk
