// Where the sweeps get C_ij from. Every source hands a wavefront lane the
// costs of VEC consecutive columns of one row, as FP64 values (columns past J
// read as +inf, which the log-domain sweeps turn into a zero plan entry).
//
//  * DenseSrc<T>: a row-major I x J matrix in HBM (FP32 or FP64), read with
//    16-byte vector loads when the row length allows it.
//  * RatesSrc<T>: a row-major rate matrix R_ij; C_ij = (1 / R_ij) / scale
//    (Sec. IV, cost choice (ii), median-normalised by the caller).
//  * GeoSrc: no matrix at all. C_ij is regenerated from device / RRH
//    positions with the downlink model of Sec. II-A:
//      R_ij = W log2(1 + SINR_ji),  SINR_ji = P G_ji / (sum_{k != j} P G_ki + N0),
//      G_ji = K0 max(d, d_min)^(-alpha) 10^(sigma X_ij / 10),
//    with X_ij a standard normal from a counter-based draw (SplitMix64 of
//    key ^ (i 2^32 + j), Box-Muller). Gains are handled relative to P K0 (the
//    received power at 1 m), and the interference of link (i, j) is taken
//    from two per-device sums prepared once per instance: S_i = sum_k pg_ik +
//    n0 and X_i = S_i - pg_{i, j1(i)} for the strongest RRH j1(i), so that
//    the dominant link never suffers the cancellation S_i - pg_ij.
//    The FP32 functor serves the fast sweeps; the FP64 functor serves the
//    polish, the exact check and the plan.
#pragma once

#include "device_common.h"

namespace otk {

__device__ __forceinline__ double pinf64() { return __builtin_huge_val(); }

// ------------------------------------------------------------ dense costs --
template <typename T>
struct DenseSrc {
    const T* C;
    int64_t ld;
    static constexpr int kTag = sizeof(T) == 4 ? 1 : 2;
    static constexpr int kVecWide = sizeof(T) == 4 ? 4 : 2;  // 16-byte loads
    static constexpr bool kCheap = true;  // re-deriving C_ij from the loaded values costs ~nothing
    static constexpr int kStageDoubles = 0;
    __device__ void stage(double*, int) const {}
    struct Row {
        const T* p;
    };
    __device__ Row row(int64_t i) const { return Row{C + i * ld}; }
    // Raw VEC-wide load of a lane's columns (issued early, converted late).
    template <int VEC>
    struct Raw {
        T v[VEC];
    };
    template <int VEC>
    __device__ __forceinline__ Raw<VEC> load(const Row& r, int col0, int J) const {
        Raw<VEC> x;
        if (col0 >= J) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x.v[v] = (T)__builtin_huge_val();
        } else if constexpr (VEC == 4 && sizeof(T) == 4) {
            // (vector loads are only used when J is a multiple of VEC, so a
            // vector is either inside the row or wholly past J)
            float4 y = *reinterpret_cast<const float4*>(r.p + col0);
            x.v[0] = y.x; x.v[1] = y.y; x.v[2] = y.z; x.v[3] = y.w;
        } else if constexpr (VEC == 2 && sizeof(T) == 8) {
            double2 y = *reinterpret_cast<const double2*>(r.p + col0);
            x.v[0] = y.x; x.v[1] = y.y;
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x.v[v] = (col0 + v < J) ? r.p[col0 + v] : (T)__builtin_huge_val();
        }
        return x;
    }
    template <bool P64, int VEC>
    __device__ __forceinline__ double cost(const Row&, const Raw<VEC>& x, int v, int64_t, int, const double*) const {
        return (double)x.v[v];
    }
    template <bool P64, int VEC>
    __device__ __forceinline__ void get(const Row& r, int64_t i, int col0, int J, const double* sm, double (&c)[VEC]) const {
        Raw<VEC> x = load<VEC>(r, col0, J);
#pragma unroll
        for (int v = 0; v < VEC; ++v) c[v] = (double)x.v[v];
    }
    __device__ __forceinline__ double at64(const Row& r, int64_t, int j, const double*) const { return (double)r.p[j]; }
};

// -------------------------------------------------------------- rate matrix --
template <typename T>
struct RatesSrc {
    const T* R;
    int64_t ld;
    double inv_scale;  // 1 / scale
    static constexpr int kTag = sizeof(T) == 4 ? 3 : 4;
    static constexpr int kVecWide = sizeof(T) == 4 ? 4 : 2;
    static constexpr bool kCheap = true;
    static constexpr int kStageDoubles = 0;
    __device__ void stage(double*, int) const {}
    struct Row {
        const T* p;
    };
    __device__ Row row(int64_t i) const { return Row{R + i * ld}; }
    template <int VEC>
    struct Raw {
        T v[VEC];
    };
    template <int VEC>
    __device__ __forceinline__ Raw<VEC> load(const Row& r, int col0, int J) const {
        Raw<VEC> x;
        if (col0 >= J) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x.v[v] = (T)0;
        } else if constexpr (VEC == 4 && sizeof(T) == 4) {
            float4 y = *reinterpret_cast<const float4*>(r.p + col0);
            x.v[0] = y.x; x.v[1] = y.y; x.v[2] = y.z; x.v[3] = y.w;
        } else if constexpr (VEC == 2 && sizeof(T) == 8) {
            double2 y = *reinterpret_cast<const double2*>(r.p + col0);
            x.v[0] = y.x; x.v[1] = y.y;
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x.v[v] = (col0 + v < J) ? r.p[col0 + v] : (T)0;
        }
        return x;
    }
    // rates of masked columns load as 0 and give C = +inf
    template <bool P64, int VEC>
    __device__ __forceinline__ double cost(const Row&, const Raw<VEC>& x, int v, int64_t, int, const double*) const {
        if constexpr (P64) return (1.0 / (double)x.v[v]) * inv_scale;
        else return (double)((float)inv_scale / (float)x.v[v]);
    }
    template <bool P64, int VEC>
    __device__ __forceinline__ void get(const Row& r, int64_t i, int col0, int J, const double* sm, double (&c)[VEC]) const {
        Raw<VEC> x = load<VEC>(r, col0, J);
#pragma unroll
        for (int v = 0; v < VEC; ++v) c[v] = (col0 + v < J) ? cost<P64, VEC>(r, x, v, i, col0 + v, sm) : pinf64();
    }
    __device__ __forceinline__ double at64(const Row& r, int64_t, int j, const double*) const {
        return (1.0 / (double)r.p[j]) * inv_scale;
    }
};

// --------------------------------------------------------------- geometry --

// SplitMix64 output for state x (Steele, Lea & Flood, 2014): add the
// golden-ratio increment, then the 30/27/31 shift-multiply mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ uint64_t link_hash(uint64_t key, int64_t i, int j) {
    return splitmix64(key ^ (((uint64_t)i << 32) + (uint64_t)(uint32_t)j));
}

// ln(1 + x) for x >= 0 in FP32 without losing the digits of small x:
// ln(u) * x / (u - 1) with u = 1 + x rounded (Goldberg's correction).
__device__ __forceinline__ float log1p_f32(float x) {
    float u = 1.0f + x;
    float l = __builtin_amdgcn_logf(u) * (float)kLn2;  // v_log_f32 is log2
    return (u == 1.0f) ? x : l * (x / (u - 1.0f));
}

// Box-Muller normal from the two 32-bit halves of h, FP32. ln(u1) is taken
// through log1p of -(1 - u1) when u1 >= 1/2, where 1 - u1 is exact.
__device__ __forceinline__ float normal_f32(uint64_t h) {
    uint32_t h1 = (uint32_t)(h >> 32), h2 = (uint32_t)h;
    bool upper = (h1 & 0x80000000u) != 0;
    float u1 = ((float)h1 + 0.5f) * 0x1p-32f;
    float v = ((float)(~h1) + 0.5f) * 0x1p-32f;  // 1 - u1
    float w = upper ? 1.0f - v : u1;
    float lw = __builtin_amdgcn_logf(w) * (float)kLn2;
    float ln_u1 = upper ? ((w == 1.0f) ? -v : lw * (-v / (w - 1.0f))) : lw;
    float u2 = ((float)h2 + 0.5f) * 0x1p-32f;
    // v_cos_f32 takes its argument in revolutions: cos(2 pi u2)
    return __builtin_sqrtf(-2.0f * ln_u1) * __builtin_amdgcn_cosf(u2);
}

__device__ __forceinline__ double normal_f64(uint64_t h) {
    uint32_t h1 = (uint32_t)(h >> 32), h2 = (uint32_t)h;
    double u1 = ((double)h1 + 0.5) * 0x1p-32;
    double u2 = ((double)h2 + 0.5) * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

struct GeoConst {
    double alpha_half;  // alpha / 2 (gain ~ (d^2)^(-alpha/2))
    double shadow_c;    // sigma log2(10) / 10: 10^(sigma X / 10) = 2^(shadow_c X)
    double dmin2;       // d_min^2
    double cscale;      // ln 2 / (W scale): C = cscale / ln(1 + SINR)
    double n0n;         // N0 / (P K0)
    uint64_t key;
};

struct GeoSrc {
    const float* dev_xy;  // I x 2
    const float* rrh_xy;  // J x 2
    const double* s_all;  // I: sum_k pg_ik + n0n
    const double* s_ex;   // I: s_all - pg_{i,j1}, summed without the strongest link
    const int* j1;        // I: strongest RRH
    GeoConst k;
    static constexpr int kTag = 5;
    static constexpr int kVecWide = 1;
    static constexpr bool kCheap = false;  // C_ij is a full functor evaluation: compute once per sweep
    static constexpr int kStageDoubles = 1;  // (x_j, y_j) as a float pair per column
    __device__ void stage(double* sm, int ncols) const {
        float2* xy = reinterpret_cast<float2*>(sm);
        for (int c = threadIdx.x; c < ncols; c += blockDim.x) xy[c] = reinterpret_cast<const float2*>(rrh_xy)[c];
    }
    struct Row {
        float x, y;
        double s_all, s_ex;
        int j1;
    };
    __device__ Row row(int64_t i) const {
        float2 p = reinterpret_cast<const float2*>(dev_xy)[i];
        return Row{p.x, p.y, s_all[i], s_ex[i], j1[i]};
    }
    __device__ __forceinline__ float cost32(const Row& r, int64_t i, int j, float2 q) const {
        float dx = r.x - q.x, dy = r.y - q.y;
        float d2 = fmaxf(fmaf(dx, dx, dy * dy), (float)k.dmin2);
        float X = normal_f32(link_hash(k.key, i, j));
        float lg = fmaf((float)k.shadow_c, X, -(float)k.alpha_half * __builtin_amdgcn_logf(d2));
        float pg = __builtin_amdgcn_exp2f(lg);
        float den = (j == r.j1) ? (float)r.s_ex : ((float)r.s_all - pg);
        float sinr = pg / den;
        return (float)k.cscale / log1p_f32(sinr);
    }
    __device__ __forceinline__ double cost64(const Row& r, int64_t i, int j, float2 q) const {
        double dx = (double)r.x - (double)q.x, dy = (double)r.y - (double)q.y;
        double d2 = fmax(dx * dx + dy * dy, k.dmin2);
        double X = normal_f64(link_hash(k.key, i, j));
        double pg = exp2(k.shadow_c * X - k.alpha_half * log2(d2));
        double den = (j == r.j1) ? r.s_ex : (r.s_all - pg);
        return k.cscale / log1p(pg / den);
    }
    template <int VEC>
    struct Raw {};
    template <int VEC>
    __device__ __forceinline__ Raw<VEC> load(const Row&, int, int) const { return Raw<VEC>{}; }
    template <bool P64, int VEC>
    __device__ __forceinline__ double cost(const Row& r, const Raw<VEC>&, int, int64_t i, int j, const double* sm) const {
        const float2 q = reinterpret_cast<const float2*>(sm)[j];
        if constexpr (P64) return cost64(r, i, j, q);
        else return (double)cost32(r, i, j, q);
    }
    template <bool P64, int VEC>
    __device__ __forceinline__ void get(const Row& r, int64_t i, int col0, int J, const double* sm,
                                        double (&c)[VEC]) const {
        const float2* xy = reinterpret_cast<const float2*>(sm);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            int j = col0 + v;
            if (j >= J) { c[v] = pinf64(); continue; }
            if constexpr (P64) c[v] = cost64(r, i, j, xy[j]);
            else c[v] = (double)cost32(r, i, j, xy[j]);
        }
    }
    __device__ __forceinline__ double at64(const Row& r, int64_t i, int j, const double* sm) const {
        return cost64(r, i, j, reinterpret_cast<const float2*>(sm)[j]);
    }
};

// -------------------------------------------------------------- Euclidean --
// C_ij = ||x_i - X_j|| / scale from device and RRH positions (Sec. IV, cost
// choice (i)): one square root per cell, in FP32 for the fast sweeps and in
// FP64 (from the same FP32 positions) for the polish, the check and the plan.
struct EuclidSrc {
    const float* dev_xy;  // I x 2
    const float* rrh_xy;  // J x 2
    double inv_scale;
    static constexpr int kTag = 6;
    static constexpr int kVecWide = 1;
    static constexpr bool kCheap = false;    // keep the computed cost for the second pass
    static constexpr int kStageDoubles = 1;  // (X_j, Y_j) as a float pair per column
    __device__ void stage(double* sm, int ncols) const {
        float2* xy = reinterpret_cast<float2*>(sm);
        for (int c = threadIdx.x; c < ncols; c += blockDim.x) xy[c] = reinterpret_cast<const float2*>(rrh_xy)[c];
    }
    struct Row {
        float x, y;
    };
    __device__ Row row(int64_t i) const {
        const float2 p = reinterpret_cast<const float2*>(dev_xy)[i];
        return Row{p.x, p.y};
    }
    __device__ __forceinline__ float cost32(const Row& r, float2 q) const {
        const float dx = r.x - q.x, dy = r.y - q.y;
        return __builtin_sqrtf(fmaf(dx, dx, dy * dy)) * (float)inv_scale;
    }
    __device__ __forceinline__ double cost64(const Row& r, float2 q) const {
        const double dx = (double)r.x - (double)q.x, dy = (double)r.y - (double)q.y;
        return sqrt(dx * dx + dy * dy) * inv_scale;
    }
    template <int VEC>
    struct Raw {};
    template <int VEC>
    __device__ __forceinline__ Raw<VEC> load(const Row&, int, int) const { return Raw<VEC>{}; }
    template <bool P64, int VEC>
    __device__ __forceinline__ double cost(const Row& r, const Raw<VEC>&, int, int64_t, int j, const double* sm) const {
        const float2 q = reinterpret_cast<const float2*>(sm)[j];
        if constexpr (P64) return cost64(r, q);
        else return (double)cost32(r, q);
    }
    template <bool P64, int VEC>
    __device__ __forceinline__ void get(const Row& r, int64_t, int col0, int J, const double* sm, double (&c)[VEC]) const {
        const float2* xy = reinterpret_cast<const float2*>(sm);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int j = col0 + v;
            if (j >= J) { c[v] = pinf64(); continue; }
            if constexpr (P64) c[v] = cost64(r, xy[j]);
            else c[v] = (double)cost32(r, xy[j]);
        }
    }
    __device__ __forceinline__ double at64(const Row& r, int64_t, int j, const double* sm) const {
        return cost64(r, reinterpret_cast<const float2*>(sm)[j]);
    }
};

}  // namespace otk
