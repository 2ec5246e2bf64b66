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
// so both GEMMs read their A operand along contiguous memory) is stored split
// into BF16 high and low parts (x = hi + lo: about 16 significant bits
// instead of BF16's 8, so that a plan concentrated on few RRHs per device
// does not inherit the 2^-9 relative rounding of a single BF16 K entry as its
// marginal error); U and V are kept in FP32 and split the same way when a
// workgroup stages them in LDS. A product is Kh Xh + Kh Xl + Kl Xh (the Kl Xl
// term is below FP32 accumulation), every product accumulating in FP32.
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
    int rows_nt;     // row tiles per workgroup of the row GEMM
    int cols_nt;     // column tiles per workgroup of the column GEMM
    const unsigned short* K;   // Ip x Jp BF16 high part, zero padded
    const unsigned short* Kt;  // K^T BF16 high part, split-major: split p's rows as a Jp x rows_per_split
                               // matrix (columns i - p rows_per_split), zero padded
    const unsigned short* Kl;  // Ip x Jp BF16 low part
    const unsigned short* Ktl; // K^T BF16 low part, the same layout
    const double* A;           // kSnapB x I marginals a_s (rows >= B unused)
    float* A32;                // kSnapB x Ip, the marginals rounded to FP32, 0 on padding
    const double* b;           // J
    float* U;                  // kSnapB x Ip, 0 on padded rows and snapshots
    float* V;                  // kSnapB x Jp, 0 on padded columns and snapshots
    unsigned short* Us;        // U split into BF16 high / low, staging layout per column split
    unsigned short* Vs;        // V split into BF16 high / low, staging layout per row-GEMM chunk
    float* Qpart;              // splits x kSnapB x Jp
    double* res;               // kSnapB: column residual of the last combined iterate
    double* mass;              // kSnapB: sum a_s
    int* ctl;                  // [0] iterations done, [1] stop, [2] max_iter, [3] result iteration;
                               // from int 8: two 64-bit decision slots (below)
    double tol;
    int cols_groups;           // (column group, split) pairs of the column GEMM
    int cols_per_xcd;          // of them per XCD (the launch has 8 times as many groups)
};

// Decision slots: the largest relative column residual of the live snapshots
// in iteration k, as the bits of a non-negative double (ordered as unsigned
// integers), gathered with atomic max in slot k % 2 by the combine of
// iteration k and read by the row pass of iteration k + 1, which also clears
// the other slot for the combine after it.
__device__ __forceinline__ unsigned long long* snap_slot(const SnapArgs& S, int k) {
    return reinterpret_cast<unsigned long long*>(S.ctl + 8) + (k & 1);
}

// K-values per staged chunk: 448 in the row GEMM (7 K-steps per wave of a
// pair: all of a 400-RRH layout at once, with 56 fragment VGPRs beside the
// staging loads for the 3 waves per SIMD of 10-wave groups), 576 in the
// column GEMM (9 K-steps per wave, 2 waves per SIMD).
constexpr int kSnapRowPS = 7;
constexpr int kSnapColPS = 9;
constexpr int kSnapRowCK = 64 * kSnapRowPS;
constexpr int kSnapColCK = 64 * kSnapColPS;

// Staging layout of a B operand (V for the row GEMM, U for the column GEMM):
// per chunk of CK K-values, a BF16 high plane and a low plane of kSnapB rows
// (snapshots) with a row stride of CK + 8 elements, chunk after chunk. A
// workgroup copies one chunk into LDS as is (256 (CK + 8) bytes, a whole
// number of KiB). In LDS a fragment read (16 lanes: snapshots t 16 .. t 16 +
// 15 at one K offset, 16 bytes each) then covers 16 distinct 4-bank groups:
// the stride is 4 (4q + 1) dwords for CK = 32 q, and 4q + 1 is odd, so
// m (4q + 1) mod 16 is distinct for m = 0 .. 15.
__host__ __device__ constexpr int snap_stage_bytes(int ck) { return 256 * (ck + 8); }
static_assert(snap_stage_bytes(kSnapRowCK) % 1024 == 0 && snap_stage_bytes(kSnapColCK) % 1024 == 0,
              "a staged chunk is copied in KiB units");
// element (s, k) of chunk c (k relative to the chunk) in a staging layout
__device__ __forceinline__ int64_t snap_stage_at(int ck, int64_t c, int s, int k, int plane) {
    return c * (snap_stage_bytes(ck) / 2) + ((int64_t)plane * 64 + s) * (ck + 8) + k;
}

// Splits x (FP32) into BF16 high and low parts.
__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

// The same split for two values at once on the gfx950 packed conversion
// (round to nearest even, as bf16_bits): the BF16 pairs (hi of a, hi of b)
// and (lo of a, lo of b), element 0 in the low half.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x2(float a, float b, unsigned& hi, unsigned& lo) {
    const bf16x2 h = {(__bf16)a, (__bf16)b};
    hi = __builtin_bit_cast(unsigned, h);
    const bf16x2 l = {(__bf16)(a - __uint_as_float(hi << 16)), (__bf16)(b - __uint_as_float(hi & 0xffff0000u))};
    lo = __builtin_bit_cast(unsigned, l);
}

// Builds the stabilised kernel as BF16 high / low parts and their
// transposes, through 32 x 32 LDS tiles: K_ij = exp2((fbar_i + gbar_j - C_ij)
// log2(e) / eps) rounded to FP32, zero outside I x J. The transposes are
// split-major (rps rows per column split, a multiple of 32), so that a
// column-GEMM workgroup reads one contiguous block per part.
__global__ __launch_bounds__(256) void k_snap_build(const float* C, int64_t ldc, int64_t I, int J, int64_t Ip, int Jp,
                                                    int64_t rps, const double* fbar, const double* gbar, double kk,
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
    const int64_t p = i0 / rps, c0 = i0 - p * rps;  // (a 32-row tile lies in one split)
    for (int r = ty; r < 32; r += 8) {
        const int64_t o = (p * Jp + j0 + r) * rps + c0 + tx;
        Kt[o] = th[tx][r];
        Ktl[o] = tl[tx][r];
    }
}

// Writes v (s, j) in FP32 and as its staged BF16 split.
__device__ __forceinline__ void snap_put_v(const SnapArgs& S, int s, int j, float v) {
    S.V[(int64_t)s * S.Jp + j] = v;
    unsigned short hi, lo;
    split_bf16(v, hi, lo);
    const int c = j / kSnapRowCK, k = j - c * kSnapRowCK;
    S.Vs[snap_stage_at(kSnapRowCK, c, s, k, 0)] = hi;
    S.Vs[snap_stage_at(kSnapRowCK, c, s, k, 1)] = lo;
}

// Sets the scaling vectors of a cold start: v = 1 on live (s, j), 0 elsewhere.
__global__ void k_snap_init(SnapArgs S) {
    const int64_t n = (int64_t)kSnapB * S.Jp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / S.Jp), j = (int)(e - (int64_t)s * S.Jp);
        snap_put_v(S, s, j, (s < S.B && j < S.J) ? 1.0f : 0.0f);
    }
    if (blockIdx.x == 0)
        for (int q = threadIdx.x; q < kSnapB; q += blockDim.x) S.res[q] = __builtin_huge_val();
}

__device__ __forceinline__ bf16x8 load8(const unsigned short* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}


// LDS of a GEMM workgroup: one staged chunk of the larger of the two chunk
// widths (the pair sums reuse it).
constexpr int kSnapChunkK = kSnapColCK;
constexpr int kSnapLdsBytes = snap_stage_bytes(kSnapChunkK);
constexpr int kSnapMaxNT = 6;  // A tiles per workgroup (2 waves each)
static_assert(kSnapLdsBytes <= 160 * 1024, "one chunk must fit the LDS of a workgroup");
static_assert(kSnapMaxNT * 4 * 64 * 16 <= kSnapLdsBytes, "the pair sums reuse the staging area");

// Raw buffer access (gfx9 resource word 3): loads at or beyond `bytes` from
// the base return 0, so a resource sized to the valid data bounds its reads.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t snap_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ bf16x8 snap_bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 snap_uload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// One workgroup's part of a stacked product D (16 NT x kSnapB) = A (16 NT x K)
// B (K x kSnapB) over the K-range [k0, k1) (multiples of 32) in chunks of
// CK = 64 PS K-values, with 2 NT waves: wave w multiplies A tile w / 2 over
// the K-steps of parity w % 2 of each chunk (at most PS), into acc (one
// 16 x 16 tile per 16 snapshots). A is read from its BF16 high / low rows (row
// stride lda elements, `live` tiles of 16 rows from Ah / Al). B comes in the
// staging layout, chunk after chunk from Bs, and is copied into LDS as is.
// Each product is Ah Bh + Ah Bl + Al Bh, accumulated in FP32; with KLO
// false the low part of A is not read (Ah Bh + Ah Bl: A in BF16 alone).
// A chunk's B copy is issued first and its A fragments after it, so that the
// copy is waited for alone and each K-step then waits for its own fragments
// only (their loads overlap the products of the steps before). `gate` runs
// after the first chunk's loads are issued; it must give every thread the
// same answer, and on true the function waits for them and returns false
// without writing anything. `pre` runs once, when the first chunk is staged.
// Offsets are 32-bit: 16 NT lda elements and the staged chunks stay far below
// 2^31 bytes.
template <int NT, int PS, bool KLO, typename Gate, typename Pre>
__device__ __forceinline__ bool snap_block(const unsigned short* Ah, const unsigned short* Al, int64_t lda, int live,
                                           const unsigned short* Bs, int64_t k0, int64_t k1, unsigned short* lds,
                                           Gate gate, Pre pre, f32x4 (&acc)[kSnapNT]) {
    constexpr int NW = 2 * NT;
    constexpr int CK = 64 * PS;
    constexpr int UNITS = snap_stage_bytes(CK) / 1024;  // KiB units of a staged chunk
    constexpr int UPW = (UNITS + NW - 1) / NW;          // units per wave
    constexpr int RU = UPW < 16 ? UPW : 16;             // units per wave in flight (groups of few waves: rounds)
    static_assert(CK <= kSnapChunkK, "chunk beyond the staging area");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = w >> 1, par = w & 1, m = lane & 15, kq = (lane >> 4) * 8;
    const bool mine = tile < live;
    const unsigned arow = (unsigned)(16 * live) * (unsigned)lda * 2u;
    const __amdgpu_buffer_rsrc_t rh = snap_rsrc(Ah, arow), rl = snap_rsrc(KLO ? Al : Ah, arow);
    const unsigned avoff = ((unsigned)(16 * tile + m) * (unsigned)lda + kq + 32 * par) * 2u;
    const unsigned nchunk = (unsigned)((k1 - k0 + CK - 1) / CK);
    const __amdgpu_buffer_rsrc_t rb = snap_rsrc(Bs, nchunk * (unsigned)snap_stage_bytes(CK));
    const unsigned short* hi = lds;
    const unsigned short* lo = lds + kSnapB * (CK + 8);
#pragma unroll
    for (int t = 0; t < kSnapNT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t c0 = k0; c0 < k1; c0 += CK) {
        const unsigned cbase = (unsigned)((c0 - k0) / CK) * (unsigned)snap_stage_bytes(CK);
        const int cw = (int)min((int64_t)CK, k1 - c0);
        const int ns = ((cw >> 5) - par + 1) >> 1;  // this wave's steps: par, par + 2, ... < cw / 32
        if (c0 != k0) __syncthreads();  // every wave is done with the previous chunk's B
        // B copy: wave w takes KiB units w, w + NW, ...; slots past the last
        // unit repeat it (the same bytes written twice to the same place),
        // so that no load or store sits behind a branch and each wait
        // counts exactly the loads before it
        u32x4 x[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u)
            x[u] = snap_uload(rb, 16u * lane, cbase + 1024u * (unsigned)min(w + NW * u, UNITS - 1));
        __builtin_amdgcn_sched_barrier(0);
        // A fragments, also without branches: steps past this wave's last one
        // repeat it, and the rows of a tile past `live` lie outside the
        // resource and read as 0 (neither is multiplied)
        bf16x8 fa[PS], fl[KLO ? PS : 1];
#pragma unroll
        for (int q = 0; q < PS; ++q) {
            const unsigned soff = (unsigned)c0 * 2u + 128u * (unsigned)min(q, ns - 1);
            fa[q] = snap_bload(rh, avoff, soff);
            if constexpr (KLO) fl[q] = snap_bload(rl, avoff, soff);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (c0 == k0 && gate()) {
            __builtin_amdgcn_s_waitcnt(0);
            return false;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) *reinterpret_cast<u32x4*>(lds + 512 * min(w + NW * u, UNITS - 1) + 8 * lane) = x[u];
        for (int r0 = RU; r0 < UPW; r0 += RU) {  // (only with few waves per group)
#pragma unroll
            for (int u = 0; u < RU; ++u)
                x[u] = snap_uload(rb, 16u * lane, cbase + 1024u * (unsigned)min(w + NW * (r0 + u), UNITS - 1));
#pragma unroll
            for (int u = 0; u < RU; ++u)
                *reinterpret_cast<u32x4*>(lds + 512 * min(w + NW * (r0 + u), UNITS - 1) + 8 * lane) = x[u];
        }
        __syncthreads();
        if (c0 == k0) pre();
        if (mine) {
#pragma clang loop unroll(full)
            for (int q = 0; q < PS; ++q)
                if (q < ns) {
                    const int kk = (2 * q + par) * 32 + kq;
                    bf16x8 bh[kSnapNT], bl[kSnapNT];
#pragma unroll
                    for (int t = 0; t < kSnapNT; ++t) {
                        const int o = (t * 16 + m) * (CK + 8) + kk;
                        bh[t] = *reinterpret_cast<const bf16x8*>(hi + o);
                        bl[t] = *reinterpret_cast<const bf16x8*>(lo + o);
                    }
#pragma unroll
                    for (int t = 0; t < kSnapNT; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[q], bh[t], acc[t], 0, 0, 0);
#pragma unroll
                    for (int t = 0; t < kSnapNT; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[q], bl[t], acc[t], 0, 0, 0);
                    if constexpr (KLO) {
#pragma unroll
                        for (int t = 0; t < kSnapNT; ++t)
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[KLO ? q : 0], bh[t], acc[t], 0, 0, 0);
                    }
                }
        }
    }
    return true;
}

// Sums the two K-parities of each A tile through LDS (reusing the staging
// area): the wave of parity p keeps snapshot tiles 2 p and 2 p + 1 and
// returns them in tot as (its part + its partner's part).
template <int NT>
__device__ __forceinline__ void snap_pair_sum(const f32x4 (&acc)[kSnapNT], unsigned short* lds, f32x4 (&tot)[2]) {
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = w >> 1, par = w & 1;
    f32x4* give = reinterpret_cast<f32x4*>(lds) + ((tile * 2 + par) * 2) * 64 + lane;
    const f32x4* take = reinterpret_cast<const f32x4*>(lds) + ((tile * 2 + (1 - par)) * 2) * 64 + lane;
    __syncthreads();  // every wave is done with the staged B
    // (branches on the wave-uniform parity, so that acc is only ever indexed
    // by constants and stays in registers)
    if (par) {
        give[0] = acc[0];
        give[64] = acc[1];
    } else {
        give[0] = acc[2];
        give[64] = acc[3];
    }
    __syncthreads();
    if (par) {
        tot[0] = acc[2] + take[0];
        tot[1] = acc[3] + take[64];
    } else {
        tot[0] = acc[0] + take[0];
        tot[1] = acc[1] + take[64];
    }
}

// Row half-step: P = K V for NT row tiles of 16 per workgroup, then
// u = a / P (0 on padded rows and snapshots), stored in FP32 and in the
// column GEMM's staging layout. The stop decision (every live snapshot's
// relative column residual of the last iterate below tol, or the iteration
// cap) is taken from scalar loads after the group's loads are issued; group
// 0 records it, or clears the decision slot of this iteration's combine.
template <int NT, bool KLO>
__global__ __launch_bounds__(128 * NT) void k_snap_rows(SnapArgs S) {
    extern __shared__ unsigned short snap_lds[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = w >> 1, par = w & 1, m = lane & 15;
    const int64_t i0 = (int64_t)blockIdx.x * (16 * NT);
    const int live = (int)min((int64_t)NT, (S.Ip - i0) / 16);
    // D: column = snapshot t 16 + m, rows i0 + 16 tile + 4 (lane / 16) + q;
    // this wave finishes snapshot tiles 2 par and 2 par + 1, whose marginals
    // are loaded before the products
    const int64_t ib = i0 + 16 * tile + (lane >> 4) * 4;
    float4 av[2] = {};
    auto load_a = [&] {
        if (tile < live)
#pragma unroll
            for (int u = 0; u < 2; ++u)
                av[u] = *reinterpret_cast<const float4*>(S.A32 + (int64_t)((2 * par + u) * 16 + m) * S.Ip + ib);
    };
    const int done = S.ctl[0];  // iterations done (advanced by the column pass)
    auto stop = [&] {
        const double r = __longlong_as_double((long long)*snap_slot(S, done));
        return S.ctl[1] != 0 || r < S.tol || done >= S.ctl[2];
    };
    auto pre = [&] {
        if (blockIdx.x == 0 && threadIdx.x == 0) *snap_slot(S, done + 1) = 0ull;
        load_a();
    };
    f32x4 acc[kSnapNT];
    if (!snap_block<NT, kSnapRowPS, KLO>(S.K + i0 * S.Jp, S.Kl + i0 * S.Jp, S.Jp, live, S.Vs, 0, S.Jp, snap_lds, stop,
                                    pre, acc)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && !S.ctl[1]) {
            S.ctl[3] = done;
            S.ctl[1] = 1;
        }
        return;
    }
    f32x4 tot[2];
    snap_pair_sum<NT>(acc, snap_lds, tot);
    if (tile >= live) return;
    // (ib .. ib + 3 lie in one column split: splits are multiples of 32 rows)
    const int64_t split = ib / S.rows_per_split;
    const int k = (int)(ib - split * S.rows_per_split);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int s = (2 * par + u) * 16 + m;
        const float a4[4] = {av[u].x, av[u].y, av[u].z, av[u].w};
        float x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float v = (float)((double)a4[q] / (double)tot[u][q]);
            x[q] = (s < S.B && ib + q < S.I) ? v : 0.0f;
        }
        *reinterpret_cast<float4*>(S.U + (int64_t)s * S.Ip + ib) = make_float4(x[0], x[1], x[2], x[3]);
        unsigned h01, l01, h23, l23;
        split_bf16x2(x[0], x[1], h01, l01);
        split_bf16x2(x[2], x[3], h23, l23);
        *reinterpret_cast<uint2*>(S.Us + snap_stage_at(kSnapColCK, split, s, k, 0)) = make_uint2(h01, h23);
        *reinterpret_cast<uint2*>(S.Us + snap_stage_at(kSnapColCK, split, s, k, 1)) = make_uint2(l01, l23);
    }
}

// Column half-step, split along i: Qpart[split] = K^T U over the split's
// rows (at most one staged chunk), for NT column tiles of 16 per workgroup.
// Workgroups go round-robin over the 8 XCDs, so group b runs on XCD b % 8:
// each XCD takes a contiguous range of (split, column group) pairs, and the
// column groups of one split share its staged U in that XCD's L2. Group 0
// of the pass counts the iteration.
template <int NT, bool KLO>
__global__ __launch_bounds__(128 * NT) void k_snap_cols(SnapArgs S) {
    extern __shared__ unsigned short snap_lds[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = w >> 1, par = w & 1, m = lane & 15;
    const int slot = blockIdx.x >> 3;
    if (slot >= S.cols_per_xcd) return;
    const int g = (blockIdx.x & 7) * S.cols_per_xcd + slot;
    if (g >= S.cols_groups) return;
    const int jgroups = S.cols_groups / S.splits;
    const int split = g / jgroups, j0 = (g - split * jgroups) * (16 * NT);
    const int live = min(NT, (S.Jp - j0) / 16);
    const int64_t r0 = (int64_t)split * S.rows_per_split;
    const int64_t r1 = min(S.Ip, r0 + S.rows_per_split);
    f32x4 acc[kSnapNT];
    const unsigned short* Bs = S.Us + (int64_t)split * (snap_stage_bytes(kSnapColCK) / 2);
    const int64_t ao = ((int64_t)split * S.Jp + j0) * S.rows_per_split;
    if (!snap_block<NT, kSnapColPS, KLO>(S.Kt + ao, S.Ktl + ao, S.rows_per_split, live, Bs, 0, r1 - r0,
                                    snap_lds, [&] { return S.ctl[1] != 0; },
                                    [&] {
                                        if (g == 0 && threadIdx.x == 0) S.ctl[0] += 1;
                                    },
                                    acc))
        return;
    f32x4 tot[2];
    snap_pair_sum<NT>(acc, snap_lds, tot);
    if (tile >= live) return;
    const int jb = j0 + 16 * tile + (lane >> 4) * 4;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int s = (2 * par + u) * 16 + m;
        float* o = S.Qpart + ((int64_t)split * kSnapB + s) * S.Jp + jb;
        *reinterpret_cast<float4*>(o) = make_float4(tot[u][0], tot[u][1], tot[u][2], tot[u][3]);
    }
}

// Sum over the column splits of one column partial (fixed order, FP64),
// R split loads in flight at a time (indices past the last split repeat it
// and are not added).
template <int R>
__device__ __forceinline__ double snap_sum_splits(const float* qp, int64_t step, int np) {
    double q = 0.0;
    for (int p = 0; p < np; p += R) {
        float x[R];
#pragma unroll
        for (int u = 0; u < R; ++u) x[u] = qp[(int64_t)min(p + u, np - 1) * step];
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (p + u < np) q += (double)x[u];
    }
    return q;
}

// Column combine, workgroup s (one per snapshot): Q = sum of the splits
// (fixed order, FP64), the column residual of the iterate (u, v_old) and
// v = b / Q (FP32 and staged). A live snapshot puts its relative residual
// (NaN counted as 0, as in a sequential fmax from 0) into this iteration's
// decision slot. The first column's split loads are issued before the stop
// flag is read (reading partials is harmless after the stop; nothing is
// stored then), so the two latencies overlap.
__global__ __launch_bounds__(512) void k_snap_combine(SnapArgs S) {
    const int s = blockIdx.x;
    __shared__ double red[8];
    double r = 0.0;
    const int64_t step = (int64_t)kSnapB * S.Jp;
    auto col_sum = [&](int j) {
        const float* qp = S.Qpart + (int64_t)s * S.Jp + j;
        return S.splits <= 16   ? snap_sum_splits<16>(qp, step, S.splits)
               : S.splits <= 32 ? snap_sum_splits<32>(qp, step, S.splits)
                                : snap_sum_splits<64>(qp, step, S.splits);
    };
    const bool first = s < S.B && (int)threadIdx.x < S.J;
    const double q0 = first ? col_sum(threadIdx.x) : 0.0;
    if (S.ctl[1]) return;  // (the same for every thread)
    for (int j = threadIdx.x; j < S.Jp; j += blockDim.x) {
        float v = 0.0f;
        if (s < S.B && j < S.J) {
            const double q = j == (int)threadIdx.x ? q0 : col_sum(j);
            r += fabs((double)S.V[(int64_t)s * S.Jp + j] * q - S.b[j]);
            v = (float)(S.b[j] / q);
        }
        snap_put_v(S, s, j, v);
    }
    r = wave_sum(r);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
        S.res[s] = t;
        if (s < S.B) {
            const double rel = fmax(0.0, t / S.mass[s]);
            __hip_atomic_fetch_max(snap_slot(S, S.ctl[0]), (unsigned long long)__double_as_longlong(rel),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
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
// padded snapshots. Also A32[s][i] = A[s][i] rounded to FP32, 0 on padding.
__global__ __launch_bounds__(256) void k_snap_mass(const double* A, int B, int64_t I, int64_t Ip, double* mass,
                                                   float* A32) {
    const int s = blockIdx.x;
    __shared__ double red[4];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < Ip; i += blockDim.x) {
        const double v = (s < B && i < I) ? A[(int64_t)s * I + i] : 0.0;
        t += v;
        A32[(int64_t)s * Ip + i] = (float)v;
    }
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
