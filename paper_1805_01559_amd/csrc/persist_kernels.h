// The FP32 phase of a single solve as ONE cooperative launch, for instances
// whose FP32 cost fits in the LDS of the whole GPU (about 40 MB on 256 CUs:
// 20000 x 400 needs 32 MB). Each workgroup (one per CU) owns a contiguous
// block of rows, fills its LDS with their costs once (read from the matrix,
// or regenerated from positions), and then runs Sinkhorn iterations
// (Sec. III-B, the alternating row and column updates of the dual
// potentials) until the device-side stop rule fires. Iteration k:
//
//   1. row update of the workgroup's rows from the LDS tile: f_i, the row
//      residual of the previous iterate and the column partials of the
//      half-iterate (FP32 exponentials, FP64 arguments, FP64 sums across
//      lanes, rows and workgroups), published to an exchange buffer;
//   2. workgroup w owns the blocks of 8 consecutive columns w, w + nb, ...:
//      it collects their partials from every workgroup, sums them in a fixed
//      order and publishes the new g_j; workgroup 0 also sums the residuals
//      and publishes the stop decision;
//   3. every workgroup collects the new g and the decision.
//
// Only O(I + J) potentials and O(nb J) partials move per iteration; the
// I x J cost is read once per launch instead of once per iteration.
//
// Exchange without fences or barriers. On this GPU the L2 of an XCD is not
// coherent with the other XCDs' L2s, and an agent-scope release writes a
// whole L2 back; so every exchanged value is stored and loaded with
// agent-scope relaxed atomics (stores that write through the L2, loads served
// at the device's coherence point), and a reader simply polls a slot until it
// holds the value of the iteration it waits for. Every exchanged double
// carries its iteration number modulo 4 in the two lowest mantissa bits (a
// relative change below 2^-50, far under the FP32 phase's own rounding), so
// slots are never emptied: buffers alternate by iteration parity, a slot's
// previous content is from two iterations earlier (a different tag), and no
// producer can get two iterations ahead of a reader (it needs every
// workgroup's contribution of the iteration in between). The exchange is laid
// out for the memory system: a producer's column partials are one contiguous
// row (whole cache lines), the owner of eight consecutive columns reads whole
// lines, and the new g and the stop decision are written in several replicas
// so that the 256 polling workgroups do not all wait on the same lines.
// Every poll is bounded: a workgroup that waits too long sets an abort word
// that releases every other poller, and the launch ends with its control
// block marked.
#pragma once

#include "kernels.h"

namespace otk {

// ----------------------------------------------------------- exchange words --
__device__ __forceinline__ void put_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get_agent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_agent(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get_agent(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Iteration tags in the two lowest mantissa bits of an exchanged double.
__device__ __forceinline__ double tag_value(double v, int k) {
    return __longlong_as_double((__double_as_longlong(v) & ~3ll) | (long long)(k & 3));
}
__device__ __forceinline__ bool has_tag(double v, int k) { return (__double_as_longlong(v) & 3) == (long long)(k & 3); }

constexpr int kColBlock = 8;        // columns per owner block: one 64-byte line of doubles
constexpr int kReplicas = 8;        // copies of the new g and of the decision word
constexpr int kMaxCoopGroups = 256; // workgroups of a cooperative launch (an owner polls 4 per thread)

// Layout of the exchange block (offsets in doubles, each part 64-byte aligned):
//   part  [2][nb][Jp]      column partials by iteration parity; a producer's
//                          row is contiguous, Jp = J rounded up to kColBlock
//   rpart [2][nb]          row-residual partials by parity (padded to a line)
//   gx    [2][kReplicas][Gs]  new g by parity, Gs = Jp rounded up to 512 (4 KiB
//                          between replicas)
//   dec   [2][kReplicas][8]   (iteration << 2) | stop, as uint64, one line per replica
//   abort [8]              uint64, nonzero once a poll gave up
struct XchLayout {
    int Jp, Gs;
    size_t part, rpart, gx, dec, abort_, total;
};
__host__ __device__ inline XchLayout persist_xch_layout(int nb, int J) {
    XchLayout L;
    L.Jp = (J + kColBlock - 1) / kColBlock * kColBlock;
    L.Gs = (L.Jp + 511) / 512 * 512;
    L.part = 0;
    L.rpart = L.part + (size_t)2 * nb * L.Jp;
    L.gx = L.rpart + ((size_t)2 * nb + 7) / 8 * 8;
    L.dec = L.gx + (size_t)2 * kReplicas * L.Gs;
    L.abort_ = L.dec + (size_t)2 * kReplicas * 8;
    L.total = L.abort_ + 8;
    return L;
}
__host__ __device__ inline size_t persist_exchange_doubles(int nb, int J) { return persist_xch_layout(nb, J).total; }

// Polls U tagged slots per lane of one wave (slot u of lane l at
// base[(u 64 + l) stride] for u 64 + l < n) until each holds tag k; absent
// slots read 0. Returns false if the wait gave up (bound reached or abort set).
template <int U>
__device__ bool poll_tagged(const double* base, int64_t stride, int n, int k, double (&x)[U], uint64_t* abort_word,
                            int max_spin) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = u * kWave + lane;
        x[u] = p < n ? get_agent(base + (int64_t)p * stride) : tag_value(0.0, k);
    }
    int spin = 0;
    for (;;) {
        bool pend = false;
#pragma unroll
        for (int u = 0; u < U; ++u) pend |= !has_tag(x[u], k);
        if (!__any(pend)) return true;
        if ((++spin & 31) == 0 && (get_agent(abort_word) != 0 || spin > max_spin)) {
            put_agent(abort_word, (uint64_t)1);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = u * kWave + lane;
            if (!has_tag(x[u], k)) x[u] = get_agent(base + (int64_t)p * stride);
        }
    }
}

// ------------------------------------------------------- persistent solve --
struct PersistArgs {
    int64_t I;
    int J;
    int Jp;   // LDS row stride of the cost tile (ncl * LPR; padding reads +inf)
    int ncl;  // cells per lane of a row: column q LPR + sub for q < ncl (<= CPL)
    int rpw;  // rows per workgroup: a whole number of wave steps
    int max_spin;
    int hold_iter;  // > 0: at iteration k0 + hold_iter of the launch no new g is published, so
                    // every wait after it ends by giving up (exercises that path); else 0
    double stall_below;
    const double* a;
    const double* b;
    double* f[2];  // iterate k lives in f[k & 1], g[k & 1]
    double* g[2];
    double* xch;   // exchange block (persist_exchange_doubles)
    Ctl* ctl;
    const SolveParams* prm;
};

// Dynamic LDS of k_persist in bytes (the layout the kernel carves): the
// tile, a slack of (CPL - ncl) LPR floats after it, then the row and column
// vectors.
// Column blocks each workgroup owns at most (workgroup w owns w, w + nb, ...).
__host__ __device__ inline int persist_owned_blocks(int nb, int J) {
    const int nblk = (J + kColBlock - 1) / kColBlock;
    return (nblk + nb - 1) / nb;
}
__host__ __device__ inline size_t persist_lds_bytes(int rpw, int J, int Jp, int waves, int slack, int nb) {
    const size_t Jr2 = (size_t)((J + 1) & ~1), Jr4 = (size_t)((J + 3) & ~3);
    return ((size_t)rpw * Jp + (size_t)slack) * 4 + Jr2 * 8 + 6 * (size_t)rpw * 8 +
           (size_t)kColBlock * persist_owned_blocks(nb, J) * 8 + (size_t)waves * Jr4 * 4;
}

// Lane layout: a row is handled by LPR lanes (32 or 64); lane `sub` owns
// columns q LPR + sub, q < CPL, so consecutive lanes read consecutive LDS
// words, each at a constant offset from the row (one address per row step).
// Every cell is processed without a branch (branches around LDS reads would
// serialise their latencies): cells q >= ncl read on into the next row of
// the tile, or into a +inf slack after it, and get g = -inf: a zero term
// (finite or +inf costs only, never a NaN). A wave advances R = 64 / LPR rows
// per step.
template <class Src, int CPL, int LPR, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_persist(PersistArgs A, Src src) {
    extern __shared__ double sm[];
    constexpr int R = kWave / LPR;
    constexpr int T = WAVES * kWave;
    const int J = A.J, Jp = A.Jp, rpw = A.rpw, ncl = A.ncl;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int sub = lane % LPR, rg = lane / LPR;
    const int nb = (int)gridDim.x, blk = (int)blockIdx.x;
    const int64_t r0 = (int64_t)blk * rpw;
    const int nrows = (int)max((int64_t)0, min((int64_t)rpw, A.I - r0));
    const int Jr2 = (J + 1) & ~1, Jr4 = (J + 3) & ~3;
    const int slack = (CPL - ncl) * LPR;  // (a multiple of 32 floats: graw stays 8-byte aligned)
    float* tile = reinterpret_cast<float*>(sm);
    double* graw = reinterpret_cast<double*>(tile + (size_t)rpw * Jp + slack);
    double* fl = graw + Jr2;   // f_i of the current iterate
    double* al = fl + rpw;     // a_i
    double* lal = al + rpw;    // ln a_i
    double* lse = lal + rpw;   // log2 sum_j 2^(g_j kk - C_ij kk) of the last row update
    double* shf = lse + rpw;   // shift of the row's exponentials in this row update
    double* rsum = shf + rpw;  // sum of those exponentials
    double* lbl = rsum + rpw;  // ln b_j of the owned columns (8 per owned block)
    const int nown = persist_owned_blocks(nb, J);
    float* red = reinterpret_cast<float*>(lbl + (size_t)kColBlock * nown);
    __shared__ Ctl cs;  // decision workgroup: the control block for the whole launch
    __shared__ double wres[WAVES];
    __shared__ double ored[WAVES][kColBlock];  // per-wave column sums of an owned block
    __shared__ uint32_t s_dec;

    const XchLayout X = persist_xch_layout(nb, J);
    double* part = A.xch + X.part;
    double* rpart = A.xch + X.rpart;
    double* gx = A.xch + X.gx;
    uint64_t* dec = reinterpret_cast<uint64_t*>(A.xch + X.dec);
    uint64_t* abort_word = reinterpret_cast<uint64_t*>(A.xch + X.abort_);
    const int rep = blk % kReplicas;  // the replica of g and of the decision this workgroup reads

    Ctl* ctl = A.ctl;
    if (ctl->stop | ctl->done) return;  // the same words for every workgroup
    const int k0 = ctl->iter;
    int has_prev = ctl->has_prev;
    const double kk = A.prm->kk, eps = A.prm->eps, inv_eps = 1.0 / A.prm->eps;
    const float kk32 = (float)kk;

    // 1. this workgroup's rows of C in FP32 (the FP64 cost rounded once);
    //    padding columns and rows past I hold +inf (a zero plan entry)
    src.stage(reinterpret_cast<double*>(red), J);  // per-column source data (positions)
    __syncthreads();
    const double* stage = reinterpret_cast<const double*>(red);
    // (the tile's cells in row-major order, eight loads in flight per thread)
    const int ntile = rpw * Jp;
    for (int e0 = 0; e0 < ntile; e0 += 8 * T) {
        typename Src::template Raw<1> raw[8];
        int lr8[8], j8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * T + (int)threadIdx.x;
            lr8[u] = e / Jp;
            j8[u] = e - lr8[u] * Jp;
            if (e < ntile && lr8[u] < nrows && j8[u] < J) raw[u] = src.template load<1>(src.row(r0 + lr8[u]), j8[u], J);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * T + (int)threadIdx.x;
            if (e < ntile) {
                float c = __builtin_huge_valf();
                if (lr8[u] < nrows && j8[u] < J) {
                    const int64_t i = r0 + lr8[u];
                    // (the FP64 cost rounded once: for costs regenerated from
                    // positions the tile then holds exactly the materialised
                    // FP32 cost, so the FP32 phase iterates on that problem)
                    c = (float)src.template cost<true, 1>(src.row(i), raw[u], 0, i, j8[u], stage);
                }
                tile[e] = c;
            }
        }
    }
    for (int e = threadIdx.x; e < slack; e += T) tile[(size_t)rpw * Jp + e] = __builtin_huge_valf();
    // 2. the rows' a_i, ln a_i and current f_i; the current g
    const double* f_in = A.f[k0 & 1];
    for (int lr = threadIdx.x; lr < rpw; lr += T) {
        const bool ok = lr < nrows;
        const double ai = ok ? A.a[r0 + lr] : 0.0;
        al[lr] = ai;
        lal[lr] = ok ? log(ai) : 0.0;
        fl[lr] = (ok && has_prev) ? f_in[r0 + lr] : 0.0;
        lse[lr] = 0.0;
    }
    const double* g_in = A.g[k0 & 1];
    for (int j = threadIdx.x; j < J; j += T) graw[j] = g_in[j];
    for (int e = threadIdx.x; e < kColBlock * nown; e += T) {
        const int j = (blk + (e / kColBlock) * nb) * kColBlock + e % kColBlock;
        lbl[e] = j < J ? log(A.b[j]) : 0.0;
    }
    // the decision workgroup (the last one: with fewer column blocks than
    // workgroups it owns none) sums the residuals and takes the stop decision
    const int dblk = nb - 1;
    if (blk == dblk && threadIdx.x == 0) cs = *ctl;
    __syncthreads();

    // g_j kk of this lane's columns (-inf past J)
    double gk[CPL];
    auto load_g = [&]() {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int j = q * LPR + sub;
            gk[q] = (q < ncl && j < J) ? graw[j] * kk : -pinf64();
        }
    };
    load_g();

    const int steps = rpw / (WAVES * R);
    int k = k0;
    bool ok = true;
    bool exact_shift = true;  // first row update of the launch: shift by the row maximum
    for (;;) {
        ++k;
        const int P = k & 1;
        // ---- 1. row update from the LDS tile
        float acc[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] = 0.0f;
        // Each row's (shift, sum) goes to LDS; after the steps one thread per
        // row finishes f_i, the next shift and the residual term (the FP64
        // logarithm and expm1 then run once per row, on every lane).
        for (int st = 0; st < steps; ++st) {
            const int lr0 = (st * WAVES + w) * R;
            const int lr = lr0 + rg;
            const bool vrow = lr < nrows;
            const float* trow = tile + (size_t)lr * Jp + sub;
            float cv[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) cv[q] = trow[q * LPR];
            // shift: the row's previous log-sum-exp (any value near the row
            // maximum keeps the FP32 exponentials in range), or the maximum
            double m = lse[lr];
            float ev[CPL];
            float s = 0.0f, s2 = 0.0f;  // even and odd cells: two shorter add chains
            bool redo = exact_shift;
            if (!redo) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const double t = fma((double)cv[q], -kk, gk[q]) - m;
                    const float e = exp2_f32((float)t);
                    ev[q] = e;
                    if (q & 1) s2 += e;
                    else s += e;
                }
            }
            double S = group_sum<LPR>((double)(s + s2));
            // a sum far from 1 means the shift drifted too far from the row
            // maximum for FP32 exponentials: redo the wave's rows with the maximum
            redo = __any(redo || (vrow && !(S >= 0x1p-100 && S <= 0x1p100)));
            if (redo) {
                // (the costs are read from LDS again: otherwise the compiler
                // keeps the FP64 arguments of every cell live across this
                // rare branch, which costs the common path its registers)
                asm volatile("" ::: "memory");
#pragma unroll
                for (int q = 0; q < CPL; ++q) cv[q] = trow[q * LPR];
                float mx = -__builtin_huge_valf();
#pragma unroll
                for (int q = 0; q < CPL; ++q) mx = fmaxf(mx, fmaf(cv[q], -kk32, (float)gk[q]));
                m = fmax((double)group_max<LPR>(mx), -1e300);
                s = 0.0f;
                s2 = 0.0f;
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const double t = fma((double)cv[q], -kk, gk[q]) - m;
                    const float e = exp2_f32((float)t);
                    ev[q] = e;
                    if (q & 1) s2 += e;
                    else s += e;
                }
                S = group_sum<LPR>((double)(s + s2));
            }
            // column partials of the half-iterate plan, pi_ij = e_ij a_i / S_i
            const float wq = vrow ? (float)al[lr] * __builtin_amdgcn_rcpf((float)S) : 0.0f;
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] = fmaf(ev[q], wq, acc[q]);
            if (sub == 0 && vrow) {
                shf[lr] = m;
                rsum[lr] = S;
            }
        }
        exact_shift = false;
        // ---- the workgroup's partials: fold the row groups of a wave (lanes
        //      sub + LPR r share columns), then the waves in FP64, published
        //      as one contiguous row of the partial buffer
        if constexpr (LPR == 32) {
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] = xor32_sum(acc[q]);
        }
        if (rg == 0) {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int j = q * LPR + sub;
                if (q < ncl && j < J) red[w * Jr4 + j] = acc[q];
            }
        }
        __syncthreads();
        // the rows of this workgroup: f_i, the next shift, the residual term
        double res = 0.0;
        for (int lr = threadIdx.x; lr < nrows; lr += T) {
            const double L2 = shf[lr] + log2(rsum[lr]);
            const double fi = eps * (lal[lr] - kLn2 * L2);
            if (has_prev) res += al[lr] * fabs(expm1((fl[lr] - fi) * inv_eps));
            fl[lr] = fi;
            lse[lr] = L2;
        }
        res = wave_sum(res);
        if (lane == 0) wres[w] = res;
        __syncthreads();
        double* prow = part + ((size_t)P * nb + blk) * X.Jp;
        for (int c = threadIdx.x; c < J; c += T) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < WAVES; ++q) t += (double)red[q * Jr4 + c];
            put_agent(prow + c, tag_value(t, k));
        }
        if (threadIdx.x == 0) {
            double r = 0.0;
#pragma unroll
            for (int q = 0; q < WAVES; ++q) r += wres[q];
            put_agent(rpart + (size_t)P * nb + blk, tag_value(r, k));
        }

        bool fail = false;
        if (blk == dblk && w == WAVES - 1) {  // residual of iterate k - 1 and the stop rule
            double x[4];
            if (!poll_tagged(rpart + (size_t)P * nb, 1, nb, k, x, abort_word, A.max_spin)) {
                fail = true;
            } else {
                double r = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) r += x[u];
                r = wave_sum(r);
                int stop = 0;
                if (lane == 0) {
                    bookkeep(&cs, r, kModeFast, A.stall_below);
                    stop = (cs.stop | cs.done) ? 1 : 0;
                }
                stop = __shfl(stop, 0, kWave);
                const uint64_t d = ((uint64_t)k << 2) | (uint64_t)stop;
                if (lane < kReplicas) put_agent(dec + ((size_t)P * kReplicas + lane) * 8, d);
            }
        }

        // ---- 2. column update of the owned blocks of kColBlock columns: thread
        //      t takes column t % 8 of producers t / 8 + 64 u (whole lines per
        //      wave), sums them in a fixed order, publishes the new g in every
        //      replica
        for (int o = blk, oi = 0; o * kColBlock < J; o += nb, ++oi) {
            static_assert(T == 512, "the owner layout assumes 512 threads");
            const int c = threadIdx.x & (kColBlock - 1), pb = threadIdx.x >> 3;
            const int j = o * kColBlock + c;
            const bool cv = j < J;
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int pr = pb + 64 * u;
                x[u] = (cv && pr < nb) ? get_agent(part + ((size_t)P * nb + pr) * X.Jp + j) : tag_value(0.0, k);
            }
            int spin = 0;
            for (;;) {
                bool pend = false;
#pragma unroll
                for (int u = 0; u < 4; ++u) pend |= !has_tag(x[u], k);
                if (!__any(pend)) break;
                if ((++spin & 31) == 0 && (get_agent(abort_word) != 0 || spin > A.max_spin)) {
                    put_agent(abort_word, (uint64_t)1);
                    fail = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (!has_tag(x[u], k)) x[u] = get_agent(part + ((size_t)P * nb + pb + 64 * u) * X.Jp + j);
            }
            // (tag bits of the partials stay in the sum: a relative change below 2^-50)
            double s = ((x[0] + x[1]) + x[2]) + x[3];
            s += dpp_d<0x128>(s);  // lanes of one wave with the same column (producers
            s = xor16_sum(s);      // pb .. pb + 7 of this wave): lane l ^ 8, l ^ 16, l ^ 32
            s = xor32_sum(s);
            if (lane < kColBlock) ored[w][lane] = s;
            if (__syncthreads_or(fail)) { fail = true; break; }
            if (threadIdx.x < kColBlock * kReplicas) {
                const int cc = threadIdx.x & (kColBlock - 1), r = threadIdx.x >> 3;
                const int jj = o * kColBlock + cc;
                if (jj < J && k - k0 != A.hold_iter) {
                    double csum = 0.0;
#pragma unroll
                    for (int q = 0; q < WAVES; ++q) csum += ored[q][cc];
                    const double gn = graw[jj] + eps * (lbl[oi * kColBlock + cc] - log(csum));
                    put_agent(gx + ((size_t)P * kReplicas + r) * X.Gs + jj, tag_value(gn, k));
                }
            }
            __syncthreads();  // ored is reused by the next block
        }
        __syncthreads();  // the combine above still reads the old g from LDS

        // ---- 3. the new g and the decision, from this workgroup's replica:
        //      every wave polls 64 columns at a time (one load per lane in
        //      flight: short poll rounds), the last wave also the decision
        bool bad = false;
        if (!fail) {
            const double* gk_new = gx + ((size_t)P * kReplicas + rep) * X.Gs;
            for (int j0 = w * kWave; j0 < J; j0 += WAVES * kWave) {
                double x[1];
                if (!poll_tagged(gk_new + j0, 1, min(J - j0, kWave), k, x, abort_word, A.max_spin)) {
                    fail = true;
                    break;
                }
                const int j = j0 + lane;
                if (j < J) {
                    graw[j] = x[0];
                    bad |= !isfinite(x[0]);
                }
            }
        }
        if (w == WAVES - 1 && lane == 0 && !fail) {
            const uint64_t* dp = dec + ((size_t)P * kReplicas + rep) * 8;
            uint64_t d = get_agent(dp);
            int spin = 0;
            while ((d >> 2) != (uint64_t)k) {
                if ((++spin & 31) == 0 && (get_agent(abort_word) != 0 || spin > A.max_spin)) {
                    put_agent(abort_word, (uint64_t)1);
                    fail = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                d = get_agent(dp);
            }
            s_dec = (uint32_t)(d & 3);
        }
        if (__syncthreads_or(fail)) { ok = false; break; }
        const bool bad_any = __syncthreads_or(bad);
        has_prev = 1;
        if (s_dec || bad_any) {
            if (bad_any && blk == dblk && threadIdx.x == 0) {
                cs.numeric_bad = 1;
                cs.done = 1;
                cs.stop = 1;
                cs.result_iter = cs.iter;
            }
            break;
        }
        load_g();
    }

    // the final iterate k: f of the rows, g (workgroup 0) and the control block
    if (ok) {
        double* fo = A.f[k & 1];
        for (int lr = threadIdx.x; lr < nrows; lr += T) fo[r0 + lr] = fl[lr];
        if (blk == 0) {
            double* go = A.g[k & 1];
            for (int j = threadIdx.x; j < J; j += T) go[j] = graw[j];
        }
    }
    if (blk == dblk && threadIdx.x == 0) {
        if (!ok) {
            cs.sync_fail = 1;
            cs.done = 1;
            cs.stop = 1;
            cs.result_iter = cs.iter;
        }
        *ctl = cs;
    }
}

// Prepares the exchange block and clears the stop flag before a persistent
// launch (grid-stride; any grid): every exchanged slot gets the tag of
// iteration k0 + 3, which neither of the first two iterations (k0 + 1,
// k0 + 2, one per buffer parity) waits for; decision and abort words start at
// zero.
static __global__ void k_xch_clear(double* xch, int nb, int J, Ctl* ctl) {
    const XchLayout X = persist_xch_layout(nb, J);
    const int k0 = ctl->iter;
    const double empty = tag_value(0.0, k0 + 3);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < X.total; q += stride)
        xch[q] = q < X.dec ? empty : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->stop = 0;
}

// Between the FP32 phase and the FP64 polish, decided on the device: the
// polish runs unless the solve is done, at max_iter, or the FP32 residual
// already met a tol above the FP32 noise threshold. The iterate is then
// moved to the buffers the host-issued launches expect: parity 0 when the
// polish runs (it starts from there), parity np & 1 when it is skipped (where
// the polish would have left it), so that the check reads parity np & 1
// either way.
static __global__ void k_polish_gate(Ctl* ctl, double* f0, double* f1, double* g0, double* g1, int64_t I, int J,
                                     double tol, double stall_below, int np) {
    const int it = ctl->iter;
    const bool met = ctl->r_last < ctl->tol_fast && tol >= stall_below;
    const bool skip = ctl->done || np <= 0 || it >= ctl->max_iter || met;
    const int want = skip ? (np & 1) : 0;
    if ((it & 1) != want) {
        const double* fs = (it & 1) ? f1 : f0;
        const double* gs = (it & 1) ? g1 : g0;
        double* fd = want ? f1 : f0;
        double* gd = want ? g1 : g0;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < I; q += stride) fd[q] = fs[q];
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < J; q += stride) gd[q] = gs[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->stop = skip ? 1 : 0;
}

// ------------------------------------------------------------ solve set-up --
// One workgroup: checks the marginals (positive and finite, equal masses),
// copies them into the solver's buffers, zeroes g for a cold start and
// writes the solve constants and the initial control block, so that a solve
// needs no host round trip before its first sweep. The masses are
// compensated sums (per-thread Neumaier sums in a fixed strided order, then a
// fixed pairwise tree of two-sum merges).
struct InitArgs {
    int64_t I;
    int J;
    int cold;
    const double* a_src;  // may equal a
    const double* b_src;  // may equal b
    double* a;
    double* b;
    double* g0;
    SolveParams* prm_out;
    Ctl* ctl_out;
    SolveParams prm;
    Ctl ctl;
    double* xch;  // exchange block zeroed by the workgroups past the first (nx doubles), or nullptr
    int64_t nx;
};

__device__ __forceinline__ void two_sum_add(double& s, double& c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Workgroup 0 checks and sums the marginals and writes the constants and
// the control block. The workgroups past it zero the cooperative exchange
// block, for a cooperative launch that starts from iteration 0: a zero slot
// carries tag 0, which neither of the launch's first two iterations (1 and
// 2, one per buffer parity) waits for, and zero decision and abort words;
// so the launch needs no clearing pass of its own.
static __global__ __launch_bounds__(1024) void k_solve_init(InitArgs A) {
    if (blockIdx.x > 0) {
        const size_t stride = (size_t)(gridDim.x - 1) * blockDim.x;
        for (size_t q = (size_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; q < (size_t)A.nx; q += stride)
            A.xch[q] = 0.0;
        return;
    }
    __shared__ double ss[2][1024], sc[2][1024];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    double sa = 0.0, ca = 0.0, sb = 0.0, cb = 0.0;
    int bad = 0;
    // (eight loads in flight per thread, then their terms in index order)
    const int64_t n8 = (int64_t)blockDim.x * 8;
    for (int64_t i0 = threadIdx.x; i0 < A.I; i0 += n8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            v[u] = i < A.I ? A.a_src[i] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            if (i < A.I) {
                if (!(v[u] > 0.0) || !isfinite(v[u])) bad |= 1;
                if (A.a != A.a_src) A.a[i] = v[u];
                two_sum_add(sa, ca, v[u]);
            }
        }
    }
    for (int j = threadIdx.x; j < A.J; j += blockDim.x) {
        const double v = A.b_src[j];
        if (!(v > 0.0) || !isfinite(v)) bad |= 2;
        if (A.b != A.b_src) A.b[j] = v;
        two_sum_add(sb, cb, v);
        if (A.cold) A.g0[j] = 0.0;
    }
    if (bad) atomicOr(&s_bad, bad);
    ss[0][threadIdx.x] = sa; sc[0][threadIdx.x] = ca;
    ss[1][threadIdx.x] = sb; sc[1][threadIdx.x] = cb;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int u = 0; u < 2; ++u) {
                double s = ss[u][threadIdx.x], c = sc[u][threadIdx.x] + sc[u][threadIdx.x + h];
                two_sum_add(s, c, ss[u][threadIdx.x + h]);
                ss[u][threadIdx.x] = s;
                sc[u][threadIdx.x] = c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ma = ss[0][0] + sc[0][0], mb = ss[1][0] + sc[1][0];
        int flags = s_bad;
        if (fabs(ma - mb) > 1e-12 * ma) flags |= 4;
        *A.prm_out = A.prm;
        Ctl c = A.ctl;
        c.mass = ma;
        c.mass_b = mb;
        c.input_bad = flags;
        if (flags) {
            c.done = 1;
            c.stop = 1;
        }
        *A.ctl_out = c;
    }
}

}  // namespace otk
