// Set-up kernels of position-based costs and of the cost median: the
// per-device interference sums of the geometry cost, the materialised FP32
// form of any cost source, and the radix-select histogram of the median.
// They run once per instance (or per admission group), not per iteration.
#pragma once

#include "kernels.h"

namespace otk {

// ------------------------------------------------------- geometry set-up --
// One wavefront per device: the strongest RRH j1 (lowest index on ties),
// s_all = sum_j pg_ij + n0n and s_ex = sum_{j != j1} pg_ij + n0n (FP64,
// per-lane index order, then a fixed butterfly).
template <int NCH>
__device__ __forceinline__ void geo_prepass_row(const GeoSrc& src, int64_t i, int J, const float2* xy, int lane,
                                                double* s_all, double* s_ex, int* j1) {
    const float2 p = reinterpret_cast<const float2*>(src.dev_xy)[i];
    double pg[NCH];
    double bv = -1.0;
    int bj = 0x7fffffff;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int j = ch * 64 + lane;
        pg[ch] = 0.0;
        if (j < J) {
            const double dx = (double)p.x - (double)xy[j].x, dy = (double)p.y - (double)xy[j].y;
            const double d2 = fmax(dx * dx + dy * dy, src.k.dmin2);
            const double X = normal_f64(link_hash(src.k.key, i, j));
            pg[ch] = exp2(src.k.shadow_c * X - src.k.alpha_half * log2(d2));
            if (pg[ch] > bv) { bv = pg[ch]; bj = j; }
        }
    }
    // argmax across lanes, lowest index on ties
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oj = __shfl_xor(bj, o, 64);
        if (ov > bv || (ov == bv && oj < bj)) { bv = ov; bj = oj; }
    }
    double sa = 0.0, se = 0.0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int j = ch * 64 + lane;
        if (j < J) {
            sa += pg[ch];
            if (j != bj) se += pg[ch];
        }
    }
    sa = wave_sum(sa);
    se = wave_sum(se);
    if (lane == 0) {
        s_all[i] = sa + src.k.n0n;
        s_ex[i] = se + src.k.n0n;
        j1[i] = bj;
    }
}

template <int NCH>
__global__ __launch_bounds__(256) void k_geo_prepass(GeoSrc src, int64_t I, int J, double* s_all, double* s_ex, int* j1) {
    __shared__ float2 xy[2048];
    for (int c = threadIdx.x; c < J; c += blockDim.x) xy[c] = reinterpret_cast<const float2*>(src.rrh_xy)[c];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (i >= I) return;
    geo_prepass_row<NCH>(src, i, J, xy, lane, s_all, s_ex, j1);
}

// Materialised FP32 cost: the FP64 functor rounded once to FP32. A lane
// evaluates kMatCols columns of its row at once (columns past J on a clamped
// index, their value discarded) so that the long dependent chains of the FP64
// functors overlap within the lane.
constexpr int kMatCols = 4;
template <class Src>
__device__ __forceinline__ void materialize_row(const Src& src, int64_t i, int J, int64_t ld, float* C,
                                                const double* sm, int lane) {
    auto row = src.row(i);
    for (int j0 = lane; j0 < ld; j0 += 64 * kMatCols) {
        double v[kMatCols];
#pragma unroll
        for (int u = 0; u < kMatCols; ++u) v[u] = src.at64(row, i, min(j0 + 64 * u, J - 1), sm);
#pragma unroll
        for (int u = 0; u < kMatCols; ++u) {
            const int j = j0 + 64 * u;
            if (j < ld) C[i * ld + j] = j < J ? (float)v[u] : __builtin_huge_valf();
        }
    }
}

template <class Src>
__global__ void k_materialize(int64_t I, int J, int64_t ld, float* C, Src src) {
    extern __shared__ double sm[];
    src.stage(sm, J);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t i = (int64_t)blockIdx.x * nw + w; i < I; i += (int64_t)gridDim.x * nw)
        materialize_row(src, i, J, ld, C, sm, lane);
}

// Radix-select histogram over the FP32 bit patterns of 1/R (positive, so the
// bit order is the value order). Pass p looks at the 11 / 11 / 10-bit digit
// below the prefix fixed by earlier passes.
template <class Src>
__global__ void k_median_hist(int64_t I, int J, int pass, uint32_t prefix, unsigned long long* hist, Src src) {
    extern __shared__ double sm[];
    __shared__ uint32_t h[2048];
    for (int q = threadIdx.x; q < 2048; q += blockDim.x) h[q] = 0;
    src.stage(sm, J);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t i = (int64_t)blockIdx.x * nw + w; i < I; i += (int64_t)gridDim.x * nw) {
        auto row = src.row(i);
        for (int j = lane; j < J; j += 64) {
            double c[1];
            src.template get<false, 1>(row, i, j, J, sm, c);
            const uint32_t u = __float_as_uint((float)c[0]);
            uint32_t bin;
            bool take;
            if (pass == 0) { take = true; bin = u >> 21; }
            else if (pass == 1) { take = (u >> 21) == prefix; bin = (u >> 10) & 0x7FFu; }
            else { take = (u >> 10) == prefix; bin = u & 0x3FFu; }
            if (take) atomicAdd(&h[bin], 1u);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2048; q += blockDim.x)
        if (h[q]) atomicAdd(&hist[q], (unsigned long long)h[q]);
}

}  // namespace otk
