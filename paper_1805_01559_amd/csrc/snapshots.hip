// Host side of the snapshot solve (ot_assoc_solve_snapshots): B traffic
// snapshots a_s over one cost C and one RRH marginal b.
//
//  1. the cost as an FP32 device matrix (materialised for rates / geometry);
//  2. a reference solve of the mean snapshot through the single-instance path,
//     whose potentials (fbar, gbar) stabilise the kernel;
//  3. K = exp((fbar + gbar - C) / eps) as BF16 high / low parts, and their
//     transposes;
//  4. the scaling iteration of all snapshots at once on the matrix cores,
//     CHUNK iterations per captured graph, stopping on the device when every
//     snapshot's column residual (of the BF16 problem) meets tol;
//  5. per snapshot, the potentials fbar + eps ln u, gbar + eps ln v and the
//     exact FP64 check of them against the cost.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ot_assoc.h"
#include "handle.h"
#include "snapshot_kernels.h"

using namespace otk;

namespace {

constexpr int kSnapChunk = 8;
constexpr int kMaxChunks = 64;  // row chunks per snapshot in the exact check
constexpr int kSnapCUs = 256;   // workgroups that fill the GPU once (one per CU)

template <bool KLO>
const void* snap_rows_kernel_t(int nt) {
    switch (nt) {
        case 1: return (const void*)k_snap_rows<1, KLO>;
        case 2: return (const void*)k_snap_rows<2, KLO>;
        case 3: return (const void*)k_snap_rows<3, KLO>;
        case 4: return (const void*)k_snap_rows<4, KLO>;
        case 5: return (const void*)k_snap_rows<5, KLO>;
        case 6: return (const void*)k_snap_rows<6, KLO>;
        default: return nullptr;
    }
}
template <bool KLO>
const void* snap_cols_kernel_t(int nt) {
    switch (nt) {
        case 1: return (const void*)k_snap_cols<1, KLO>;
        case 2: return (const void*)k_snap_cols<2, KLO>;
        case 3: return (const void*)k_snap_cols<3, KLO>;
        case 4: return (const void*)k_snap_cols<4, KLO>;
        default: return nullptr;
    }
}
// (klo: K in BF16 high and low parts; else in BF16 alone)
const void* snap_rows_kernel(int nt, bool klo) { return klo ? snap_rows_kernel_t<true>(nt) : snap_rows_kernel_t<false>(nt); }
const void* snap_cols_kernel(int nt, bool klo) { return klo ? snap_cols_kernel_t<true>(nt) : snap_cols_kernel_t<false>(nt); }

size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct SnapState {
    int device = 0;
    // capacity of the buffers
    int64_t cap_I = 0;
    int cap_J = 0, cap_splits = 0;
    char* mem = nullptr;
    size_t bytes = 0;
    SnapArgs S{};
    double* fbar = nullptr;
    double* gbar = nullptr;
    double* abar = nullptr;   // device copy of the mean marginal
    double* bdev = nullptr;
    float* Cconv = nullptr;   // converted / materialised cost (I x J) when needed
    double* F = nullptr;      // kSnapB x I potentials f_s
    double* G = nullptr;      // kSnapB x J potentials g_s
    double* ccol = nullptr;   // check: kSnapB x kMaxChunks x J column partials
    double* cstat = nullptr;  // check: kSnapB x kMaxChunks x 5 row statistics
    double* cout = nullptr;   // check: kSnapB x 8 results
    int* ctl_h = nullptr;     // pinned mirror of S.ctl
    hipGraphExec_t graph = nullptr;
    SnapArgs graph_args{};
    double eps = 0.0;
    bool valid = false;       // a finished solve is held
    std::vector<ot_assoc_result> res;
    std::vector<double> mass;
};

void snap_state_destroy(SnapState* s) {
    if (!s) return;
    hipSetDevice(s->device);
    if (s->graph) hipGraphExecDestroy(s->graph);
    if (s->mem) hipFree(s->mem);
    if (s->ctl_h) hipHostFree(s->ctl_h);
    delete s;
}

namespace {

ot_status sfail(ot_assoc* h, ot_status st, const std::string& m) {
    h->err = m;
    return st;
}

#define SCHK(call)                                                                                        \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return sfail(h, e_ == hipErrorOutOfMemory ? OT_ENOMEM : OT_EDEVICE,                           \
                         std::string(#call " failed: ") + hipGetErrorString(e_));                         \
    } while (0)

// Converts a dense or rate matrix (device, FP32 / FP64, row stride lds) into
// an FP32 cost matrix (I x J).
template <typename T, int KIND>
__global__ void k_snap_conv(const T* src, int64_t I, int J, int64_t lds, double inv_scale, float* dst) {
    const int64_t n = I * J;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / J;
        const double x = (double)src[i * lds + (e - i * J)];
        dst[e] = KIND == 0 ? (float)x : (float)((1.0 / x) * inv_scale);
    }
}

// (Re)allocates the snapshot buffers for I x J.
ot_status snap_reserve(ot_assoc* h, SnapState* s, int64_t I, int J) {
    const int64_t Ip = (int64_t)up((size_t)I, 32);
    const int Jp = (int)up((size_t)J, 32);
    // Workgroups hold one LDS chunk each, one per CU: the row GEMM takes
    // enough row tiles per group for about one group per CU (at most
    // kSnapMaxNT); the column GEMM groups 4 column tiles and splits the rows
    // so that all (column group, split) pairs fill the CUs once, at least 64
    // rows (one K-step per wave of a pair) and at most one staged chunk per
    // split
    const int64_t tiles_i = Ip / 16;
    const int rows_nt = (int)std::min<int64_t>(kSnapMaxNT, std::max<int64_t>(1, (tiles_i + kSnapCUs - 1) / kSnapCUs));
    const int tiles_j = Jp / 16;
    const int cols_nt = std::min(4, tiles_j);
    const int jgroups = (tiles_j + cols_nt - 1) / cols_nt;
    const int64_t target = std::max(1, kSnapCUs / jgroups);
    const int64_t rps = std::min<int64_t>(kSnapColCK, std::max<int64_t>(64, (int64_t)up((size_t)((Ip + target - 1) / target), 32)));
    const int splits = (int)((Ip + rps - 1) / rps);
    if (s->mem && I <= s->cap_I && J <= s->cap_J && splits <= s->cap_splits && Ip == s->S.Ip && Jp == s->S.Jp) {
        s->S.I = I;
        s->S.J = J;
        return OT_OK;
    }
    if (s->graph) hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    if (s->mem) hipFree(s->mem);
    s->mem = nullptr;
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> parts;
    SnapArgs& S = s->S;
    S = SnapArgs{};
    auto add = [&](void** p, size_t b) { parts.push_back({p, b}); };
    add((void**)&S.K, 2 * (size_t)Ip * Jp);
    add((void**)&S.Kt, 2 * (size_t)Jp * splits * rps);
    add((void**)&S.Kl, 2 * (size_t)Ip * Jp);
    add((void**)&S.Ktl, 2 * (size_t)Jp * splits * rps);
    add((void**)&S.A, 8 * (size_t)kSnapB * I);
    add((void**)&S.A32, 4 * (size_t)kSnapB * Ip);
    add((void**)&S.b, 8 * (size_t)J);
    add((void**)&S.U, 4 * (size_t)kSnapB * Ip);
    add((void**)&S.V, 4 * (size_t)kSnapB * Jp);
    const size_t us_bytes = (size_t)splits * snap_stage_bytes(kSnapColCK);
    const size_t vs_bytes = (size_t)((Jp + kSnapRowCK - 1) / kSnapRowCK) * snap_stage_bytes(kSnapRowCK);
    add((void**)&S.Us, us_bytes);
    add((void**)&S.Vs, vs_bytes);
    add((void**)&S.Qpart, 4 * (size_t)splits * kSnapB * Jp);
    add((void**)&S.res, 8 * (size_t)kSnapB);
    add((void**)&S.mass, 8 * (size_t)kSnapB);
    add((void**)&S.ctl, 64);
    add((void**)&s->fbar, 8 * (size_t)I);
    add((void**)&s->gbar, 8 * (size_t)J);
    add((void**)&s->abar, 8 * (size_t)I);
    add((void**)&s->bdev, 8 * (size_t)J);
    add((void**)&s->Cconv, 4 * (size_t)I * J);
    add((void**)&s->F, 8 * (size_t)kSnapB * I);
    add((void**)&s->G, 8 * (size_t)kSnapB * J);
    add((void**)&s->ccol, 8 * (size_t)kSnapB * kMaxChunks * J);
    add((void**)&s->cstat, 8 * (size_t)kSnapB * kMaxChunks * 5);
    add((void**)&s->cout, 8 * (size_t)kSnapB * 8);
    for (auto& p : parts) off += up(p.second, 256);
    SCHK(otk_host::dev_malloc((void**)&s->mem, off));
    off = 0;
    for (auto& p : parts) {
        *p.first = s->mem + off;
        off += up(p.second, 256);
    }
    s->bytes = off;
    // the staging layouts' padding is never written by the iteration: zero
    // it once (it is never read either)
    SCHK(hipMemsetAsync(S.Us, 0, us_bytes, h->stream));
    SCHK(hipMemsetAsync(S.Vs, 0, vs_bytes, h->stream));
    if (!s->ctl_h) SCHK(hipHostMalloc(&s->ctl_h, 64));
    S.I = I;
    S.Ip = Ip;
    S.J = J;
    S.Jp = Jp;
    S.splits = splits;
    S.rows_per_split = rps;
    S.rows_nt = rows_nt;
    S.cols_nt = cols_nt;
    S.cols_groups = jgroups * splits;
    S.cols_per_xcd = (S.cols_groups + 7) / 8;
    s->cap_I = I;
    s->cap_J = J;
    s->cap_splits = splits;
    return OT_OK;
}

ot_status snap_capture(ot_assoc* h, SnapState* s) {
    if (s->graph && std::memcmp(&s->graph_args, &s->S, sizeof(SnapArgs)) == 0) return OT_OK;
    if (s->graph) hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    SnapArgs S = s->S;
    const bool klo = h->opt.snapshot_k_split != 0;
    const void* rows_k = snap_rows_kernel(S.rows_nt, klo);
    const void* cols_k = snap_cols_kernel(S.cols_nt, klo);
    if (!rows_k || !cols_k) return sfail(h, OT_EINVAL, "no snapshot kernel for this shape");
    SCHK(hipFuncSetAttribute(rows_k, hipFuncAttributeMaxDynamicSharedMemorySize, kSnapLdsBytes));
    SCHK(hipFuncSetAttribute(cols_k, hipFuncAttributeMaxDynamicSharedMemorySize, kSnapLdsBytes));
    // (Ip and Jp are multiples of 32, so every tile of 16 is whole)
    const dim3 rows_grid((unsigned)((S.Ip / 16 + S.rows_nt - 1) / S.rows_nt));
    const dim3 cols_grid((unsigned)(8 * S.cols_per_xcd));
    void* args[] = {&S};
    hipGraph_t g = nullptr;
    SCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < kSnapChunk; ++t) {
        (void)hipLaunchKernel(rows_k, rows_grid, dim3(128 * S.rows_nt), args, kSnapLdsBytes, h->stream);
        (void)hipLaunchKernel(cols_k, cols_grid, dim3(128 * S.cols_nt), args, kSnapLdsBytes, h->stream);
        hipLaunchKernelGGL(k_snap_combine, dim3(kSnapB), dim3(512), 0, h->stream, S);
    }
    hipError_t e1 = hipStreamEndCapture(h->stream, &g);
    if (e1 != hipSuccess) return sfail(h, OT_EDEVICE, std::string("capture failed: ") + hipGetErrorString(e1));
    hipError_t e2 = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) return sfail(h, OT_EDEVICE, std::string("instantiate failed: ") + hipGetErrorString(e2));
    s->graph_args = S;
    return OT_OK;
}

}  // namespace

extern "C" {

ot_status ot_assoc_solve_snapshots(ot_assoc* h, const ot_cost_desc* cost, int B, const double* A, const double* b,
                                   double eps, double tol, int32_t max_iter, ot_assoc_result* out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!cost || !A || !b) return sfail(h, OT_EINVAL, "cost, snapshots or b is NULL");
    if (B < 1 || B > kSnapB) return sfail(h, OT_EINVAL, "B must be in 1..64");
    if (!(eps > 0.0) || !std::isfinite(eps) || !(tol >= 0.0) || max_iter < 1)
        return sfail(h, OT_EINVAL, "bad eps, tol or max_iter");
    const int64_t I = cost->I, J64 = cost->J;
    if (I < 1 || J64 < 1 || I > h->I_max || J64 > h->J_max) return sfail(h, OT_EINVAL, "instance outside the handle's limits");
    const int J = (int)J64;
    if (hipSetDevice(h->device) != hipSuccess) return sfail(h, OT_EDEVICE, "hipSetDevice failed");
    if (!h->snap) {
        h->snap = new SnapState();
        h->snap->device = h->device;
    }
    SnapState* s = h->snap;
    s->valid = false;
    if (ot_status st = snap_reserve(h, s, I, J)) return st;
    SnapArgs& S = s->S;
    S.B = B;
    S.tol = tol;
    // snapshot marginals into the device buffer, their mean, masses and a
    // validity flag on the device (one small read-back)
    const ot_mem mem = (cost->kind == OT_COST_GEOMETRY || cost->kind == OT_COST_EUCLID) ? OT_MEM_DEVICE : cost->mem;
    const hipMemcpyKind kin = mem == OT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    SCHK(hipMemcpyAsync((double*)S.A, A, sizeof(double) * (size_t)B * I, kin, h->stream));
    SCHK(hipMemcpyAsync(s->bdev, b, sizeof(double) * J, kin, h->stream));
    SCHK(hipMemsetAsync(S.ctl + 4, 0, sizeof(int), h->stream));
    hipLaunchKernelGGL(k_snap_mean, dim3((unsigned)std::min<int64_t>(1024, (I + 255) / 256)), dim3(256), 0, h->stream,
                       (const double*)S.A, B, I, s->abar, S.ctl + 4);
    hipLaunchKernelGGL(k_snap_mass, dim3(kSnapB), dim3(256), 0, h->stream, (const double*)S.A, B, I, S.Ip, S.mass,
                       S.A32);
    std::vector<double> mass64(kSnapB), bh(J);
    SCHK(hipMemcpyAsync(mass64.data(), S.mass, sizeof(double) * kSnapB, hipMemcpyDeviceToHost, h->stream));
    SCHK(hipMemcpyAsync(bh.data(), s->bdev, sizeof(double) * J, hipMemcpyDeviceToHost, h->stream));
    SCHK(hipMemcpyAsync(s->ctl_h + 4, S.ctl + 4, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    SCHK(hipStreamSynchronize(h->stream));
    if (s->ctl_h[4]) return sfail(h, OT_EINVAL, "snapshot marginals must be positive and finite");
    for (double v : bh)
        if (!(v > 0.0) || !std::isfinite(v)) return sfail(h, OT_EINVAL, "b must be positive and finite");
    s->mass.assign(mass64.begin(), mass64.begin() + B);
    // 1. the cost as an FP32 device matrix
    const float* C = nullptr;
    int64_t ldc = J;
    if (cost->kind == OT_COST_DENSE && cost->mem == OT_MEM_DEVICE && cost->dtype == OT_F32) {
        C = (const float*)cost->data;
        ldc = cost->ld ? cost->ld : J;
    } else if (cost->kind == OT_COST_GEOMETRY || cost->kind == OT_COST_RATES || cost->kind == OT_COST_EUCLID) {
        ot_status st = ot_assoc_materialize_cost(h, cost, s->Cconv);
        if (st) return st;
        C = s->Cconv;
    } else {
        const int64_t lds = cost->ld ? cost->ld : J;
        const size_t esz = cost->dtype == OT_F32 ? 4 : 8;
        const void* src = cost->data;
        void* tmp = nullptr;
        if (cost->mem == OT_MEM_HOST) {
            SCHK(otk_host::dev_malloc((void**)&tmp, esz * (size_t)(I * lds)));
            SCHK(hipMemcpyAsync(tmp, cost->data, esz * (size_t)(I * lds), hipMemcpyHostToDevice, h->stream));
            src = tmp;
        }
        const unsigned grid = (unsigned)std::min<int64_t>(4096, (I * J + 255) / 256);
        if (cost->dtype == OT_F32)
            hipLaunchKernelGGL((k_snap_conv<float, 0>), dim3(grid), dim3(256), 0, h->stream, (const float*)src, I, J, lds, 1.0, s->Cconv);
        else
            hipLaunchKernelGGL((k_snap_conv<double, 0>), dim3(grid), dim3(256), 0, h->stream, (const double*)src, I, J, lds, 1.0, s->Cconv);
        if (tmp) {
            SCHK(hipStreamSynchronize(h->stream));
            hipFree(tmp);
        }
        C = s->Cconv;
    }
    // 2. reference solve of the mean snapshot
    ot_cost_desc dd{};
    dd.kind = OT_COST_DENSE;
    dd.I = I;
    dd.J = J;
    dd.mem = OT_MEM_DEVICE;
    dd.dtype = OT_F32;
    dd.data = C;
    dd.ld = ldc == J ? 0 : ldc;
    ot_assoc_result ref{};
    // (the reference only conditions the kernel, and the snapshots differ
    // from their mean by far more than its residual: at 20000 x 400 x 64,
    // tol 1e-3 instead of 1e-6 leaves the snapshot iterations and their
    // FP64-checked violations as they were and saves a quarter millisecond)
    ot_status st = ot_assoc_solve(h, &dd, s->abar, s->bdev, eps, 1e-3, std::max(2000, max_iter), 0, &ref);
    if (st < 0) return st;
    if ((st = ot_assoc_potentials(h, s->fbar, s->gbar, OT_MEM_DEVICE))) return st;
    // 3. stabilised kernel as BF16 high / low parts and their transposes
    const double kk = std::log2(std::exp(1.0)) / eps;
    hipLaunchKernelGGL(k_snap_build, dim3((unsigned)(S.Jp / 32), (unsigned)(S.Ip / 32)), dim3(256), 0, h->stream, C, ldc,
                       I, J, S.Ip, S.Jp, S.rows_per_split, (const double*)s->fbar, (const double*)s->gbar, kk, (unsigned short*)S.K,
                       (unsigned short*)S.Kt, (unsigned short*)S.Kl, (unsigned short*)S.Ktl);
    // 4. the snapshot iteration
    SCHK(hipMemcpyAsync((double*)S.b, s->bdev, sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream));
    s->ctl_h[0] = 0;
    s->ctl_h[1] = 0;
    s->ctl_h[2] = max_iter;
    s->ctl_h[3] = 0;
    s->ctl_h[4] = 0;
    // decision slots: +inf for the first row pass, 0 for the first combine
    const unsigned long long slots[2] = {0x7ff0000000000000ull, 0ull};
    std::memcpy(s->ctl_h + 8, slots, sizeof(slots));
    SCHK(hipMemcpyAsync(S.ctl, s->ctl_h, 12 * sizeof(int), hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(k_snap_init, dim3(64), dim3(256), 0, h->stream, S);
    SCHK(hipGetLastError());
    if ((st = snap_capture(h, s))) return st;
    hipEvent_t e0, e1;
    SCHK(hipEventCreate(&e0));
    SCHK(hipEventCreate(&e1));
    SCHK(hipEventRecord(e0, h->stream));
    const long max_chunks = max_iter / kSnapChunk + 2;
    for (long c = 0; c < max_chunks; ++c) {
        SCHK(hipGraphLaunch(s->graph, h->stream));
        SCHK(hipMemcpyAsync(s->ctl_h, S.ctl, 4 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        SCHK(hipStreamSynchronize(h->stream));
        if (s->ctl_h[1]) break;
    }
    SCHK(hipEventRecord(e1, h->stream));
    SCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    const bool converged = s->ctl_h[1] != 0 && s->ctl_h[3] < max_iter;
    const int iters = s->ctl_h[1] ? s->ctl_h[3] : s->ctl_h[0];
    std::vector<double> resid(kSnapB);
    SCHK(hipMemcpy(resid.data(), S.res, sizeof(double) * kSnapB, hipMemcpyDeviceToHost));
    // 5. potentials of every snapshot and their exact FP64 check, in three
    //    launches and one read-back
    const dim3 pg(64, (unsigned)B);
    hipLaunchKernelGGL(k_snap_all_potentials, pg, dim3(256), 0, h->stream, S, (const double*)s->fbar,
                       (const double*)s->gbar, eps, s->F, s->G);
    const int nchunk = (int)std::min<int64_t>({(int64_t)kMaxChunks, (int64_t)std::max(1, 512 / B), (I + 7) / 8});
    const int64_t rpc = (I + nchunk - 1) / nchunk;
    const int nch = (J + 63) / 64;
    const dim3 cg((unsigned)nchunk, (unsigned)B);
    if (nch <= 2)
        hipLaunchKernelGGL(k_snap_check<2>, cg, dim3(512), sizeof(double) * 4 * 2 * 64, h->stream, C, ldc, I, J, rpc,
                           (const double*)S.A, (const double*)s->F, (const double*)s->G, kk, s->ccol, s->cstat);
    else if (nch <= 8)
        hipLaunchKernelGGL(k_snap_check<8>, cg, dim3(512), sizeof(double) * 4 * 8 * 64, h->stream, C, ldc, I, J, rpc,
                           (const double*)S.A, (const double*)s->F, (const double*)s->G, kk, s->ccol, s->cstat);
    else
        hipLaunchKernelGGL(k_snap_check<32>, cg, dim3(512), sizeof(double) * 4 * 32 * 64, h->stream, C, ldc, I, J,
                           rpc, (const double*)S.A, (const double*)s->F, (const double*)s->G, kk, s->ccol, s->cstat);
    hipLaunchKernelGGL(k_snap_check_finish, dim3((unsigned)B), dim3(256), 0, h->stream, nchunk, J,
                       (const double*)S.b, (const double*)s->G, (const double*)s->ccol, (const double*)s->cstat,
                       (const double*)S.mass, eps, s->cout);
    SCHK(hipGetLastError());
    std::vector<double> chk((size_t)kSnapB * 8);
    SCHK(hipMemcpyAsync(chk.data(), s->cout, sizeof(double) * 8 * B, hipMemcpyDeviceToHost, h->stream));
    SCHK(hipStreamSynchronize(h->stream));
    s->res.assign(B, ot_assoc_result{});
    s->eps = eps;
    for (int q = 0; q < B; ++q) {
        ot_assoc_result& r = s->res[q];
        const double* c8 = chk.data() + (size_t)q * 8;
        r.marginal_violation = c8[0];
        r.objective = c8[1];
        r.reg_objective = c8[2];
        r.dual_objective = c8[3];
        r.iterations = iters;
        r.fp64_iterations = 0;
        const bool met = resid[q] / s->mass[q] < tol;
        r.status = !std::isfinite(r.marginal_violation) ? OT_ENUMERIC : (converged || met) ? OT_OK : OT_WARN_MAXITER;
        // the exact FP64 check of the returned potentials did not confirm tol
        // (the BF16 problem met it; its rounding moved the FP64 marginals)
        r.flags = (r.marginal_violation >= tol) ? OT_RESULT_CHECK_ABOVE_TOL : 0;
        r.seconds = ms * 1e-3;
        if (out) out[q] = r;
    }
    s->valid = true;
    ot_status worst = OT_OK;
    for (auto& r : s->res) {
        if (r.status < 0) worst = (ot_status)r.status;
        else if (r.status > 0 && worst == OT_OK) worst = (ot_status)r.status;
    }
    if (worst < 0) h->err = "a snapshot failed numerically";
    return worst;
}

ot_status ot_assoc_snapshot_potentials(ot_assoc* h, int s_idx, double* f, double* g, ot_mem mem) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    SnapState* s = h->snap;
    if (!s || !s->valid) return sfail(h, OT_ESTATE, "no snapshot solve to read from");
    if (s_idx < 0 || s_idx >= s->S.B) return sfail(h, OT_EINVAL, "snapshot index out of range");
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) return sfail(h, OT_EINVAL, "bad memory space");
    if (hipSetDevice(h->device) != hipSuccess) return sfail(h, OT_EDEVICE, "hipSetDevice failed");
    const hipMemcpyKind k = mem == OT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (f) SCHK(hipMemcpyAsync(f, s->F + (size_t)s_idx * s->S.I, sizeof(double) * s->S.I, k, h->stream));
    if (g) SCHK(hipMemcpyAsync(g, s->G + (size_t)s_idx * s->S.J, sizeof(double) * s->S.J, k, h->stream));
    SCHK(hipStreamSynchronize(h->stream));
    return OT_OK;
}

}  // extern "C"
