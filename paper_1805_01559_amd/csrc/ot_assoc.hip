// Host runtime and C ABI of the association solver (include/ot_assoc.h).
//
// A solve runs three phases on one HIP stream:
//   fast    FP32-exponential sweeps until the residual meets tol or stalls at
//           the FP32 noise floor. When the instance's FP32 cost fits in the
//           LDS of the GPU this is ONE cooperative launch (persist_kernels.h)
//           that keeps the cost on chip; otherwise the sweeps are captured in
//           HIP graphs CHUNK iterations at a time, and the combine kernel
//           stops the chunk on the device;
//   polish  a few FP64 sweeps, then an exact FP64 check of the iterate;
//   exact   (only if the check misses tol) FP64 sweeps until an FP64 iterate
//           meets tol, then the check again.
// Inputs are checked on the device (the verdict travels in the control
// block). With the cooperative launch a solve has a single host wait before
// the exact phase; the chunked form reads the control block once per chunk,
// one chunk behind the device, so there is no host round trip per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ot_assoc.h"
#include "handle.h"
#include "kernels.h"
#include "persist_kernels.h"
#include "assoc_kernels.h"
#include "setup_kernels.h"
#include "launchers.h"

using namespace otk;

// the launchers' kernels are instantiated in launch_dense.hip, launch_rates.hip
// and launch_geo.hip (compiled in parallel)
OT_LAUNCHERS(extern, DenseSrc<float>)
OT_LAUNCHERS(extern, DenseSrc<double>)
OT_LAUNCHERS(extern, RatesSrc<float>)
OT_LAUNCHERS(extern, RatesSrc<double>)
OT_LAUNCHERS(extern, GeoSrc)
OT_LAUNCHERS(extern, EuclidSrc)

using otk_launch::kMaxNb;

namespace {

// handle-less errors (ot_assoc_create, ot_assoc_solve_static): a fixed
// per-thread buffer, so that reporting one allocates nothing
thread_local char g_noh_err[512];
thread_local int g_test_hold = 0;  // ot_assoc_test_hold_exchange


constexpr int kMaxJ = 2048;     // RRHs per instance
constexpr int kGraphCache = 24;

using otk_host::GraphEntry;

// ------------------------------------------------------------- workspace --
// The handle's fixed device buffers, in one block; each starts on a
// kWsAlign-byte boundary.
constexpr int kWsAlign = 256;
enum {
    kWsA, kWsLa, kWsB, kWsF0, kWsF1, kWsG0, kWsG1, kWsColPart, kWsResPart, kWsStatPart, kWsCpart, kWsCtl, kWsPrm,
    kWsBad, kWsHist, kWsXch, kWsXyDev, kWsXyRrh, kWsSAll, kWsSEx, kWsJ1, kWsLoads, kWsWork, kWsCount
};
struct WsLayout {
    size_t off[kWsCount];
    size_t total;
};
// Bytes of the per-call work region: the plan's and the timers' copies of
// the potentials (I_max + J_max doubles each).
inline size_t ws_work_bytes(int64_t I_max, int64_t J_max) { return sizeof(double) * 2 * (size_t)(I_max + J_max); }

void ws_layout(int64_t I_max, int64_t J_max, WsLayout& L) {
    const size_t I8 = sizeof(double) * (size_t)I_max, J8 = sizeof(double) * (size_t)J_max;
    size_t sz[kWsCount];
    sz[kWsA] = I8; sz[kWsLa] = I8; sz[kWsB] = J8;
    sz[kWsF0] = I8; sz[kWsF1] = I8; sz[kWsG0] = J8; sz[kWsG1] = J8;
    sz[kWsColPart] = (size_t)kMaxNb * J8;
    sz[kWsResPart] = sizeof(double) * kMaxNb;
    sz[kWsStatPart] = sizeof(double) * 5 * kMaxNb;
    sz[kWsCpart] = sizeof(double) * 2 * ((kMaxJ + kColsPerWg - 1) / kColsPerWg);
    sz[kWsCtl] = sizeof(Ctl);
    sz[kWsPrm] = sizeof(SolveParams);
    sz[kWsBad] = sizeof(int);
    sz[kWsHist] = sizeof(unsigned long long) * 2048;
    sz[kWsXch] = sizeof(double) * persist_exchange_doubles(kMaxCoopGroups, (int)J_max);
    sz[kWsXyDev] = sizeof(float) * 2 * (size_t)I_max;
    sz[kWsXyRrh] = sizeof(float) * 2 * (size_t)J_max;
    sz[kWsSAll] = I8; sz[kWsSEx] = I8;
    sz[kWsJ1] = sizeof(int) * (size_t)I_max;
    sz[kWsLoads] = J8;
    sz[kWsWork] = ws_work_bytes(I_max, J_max);
    size_t o = 0;
    for (int k = 0; k < kWsCount; ++k) {
        L.off[k] = o;
        o += (sz[k] + kWsAlign - 1) / kWsAlign * kWsAlign;
    }
    L.total = o;
}

std::atomic<long long> g_dev_allocs{0};

// Points the handle's fixed buffers into the block `ws` (layout wl).
void carve_ws(ot_assoc* h, void* ws, const WsLayout& wl) {
    {
        char* base = (char*)ws;
        auto at = [&](int k) { return (void*)(base + wl.off[k]); };
        h->a = (double*)at(kWsA);
        h->la = (double*)at(kWsLa);
        h->b = (double*)at(kWsB);
        h->f[0] = (double*)at(kWsF0);
        h->f[1] = (double*)at(kWsF1);
        h->g[0] = (double*)at(kWsG0);
        h->g[1] = (double*)at(kWsG1);
        h->col_part = (double*)at(kWsColPart);
        h->res_part = (double*)at(kWsResPart);
        h->stat_part = (double*)at(kWsStatPart);
        h->cpart = (double*)at(kWsCpart);
        h->ctl = (Ctl*)at(kWsCtl);
        h->prm = (SolveParams*)at(kWsPrm);
        h->bad = (int*)at(kWsBad);
        h->hist = (unsigned long long*)at(kWsHist);
        h->xch = (double*)at(kWsXch);
        h->xy_dev = (float*)at(kWsXyDev);
        h->xy_rrh = (float*)at(kWsXyRrh);
        h->s_all = (double*)at(kWsSAll);
        h->s_ex = (double*)at(kWsSEx);
        h->j1 = (int*)at(kWsJ1);
        h->loads = (double*)at(kWsLoads);
        h->work = at(kWsWork);
    }
}

}  // namespace

namespace otk_host {
hipError_t dev_malloc(void** p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) g_dev_allocs.fetch_add(1, std::memory_order_relaxed);
    return e;
}
hipError_t dev_free(void* p) { return hipFree(p); }
}  // namespace otk_host


namespace {

ot_status fail(ot_assoc* h, ot_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h && h->err_fixed) std::memcpy(h->err_fixed, buf, sizeof buf);
    else if (h) h->err = buf;
    else std::memcpy(g_noh_err, buf, sizeof buf);
    return st;
}

#define HIPCHK(h, call)                                                                                  \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return fail((h), (e_ == hipErrorOutOfMemory) ? OT_ENOMEM : OT_EDEVICE, "%s failed: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                               \
    } while (0)

using namespace otk_launch;

// Default grid of the iteration kernel: one full wave of resident workgroups
// (as many as fit on every CU at once, at most kMaxNb partial rows and no more
// than the rows need), so that no workgroup waits for a second round.
template <class Src, bool P64>
void fit_grid(const ot_assoc* h, int64_t I, Shape& s) {
    if (h->opt.sweep_blocks > 0 || h->num_cu <= 0) return;
    int occ = 0;
    g_occupancy_query = &occ;
    IterArgs A{};
    Src src{};
    const bool known = launch_iter<Src, P64>(s, A, src, nullptr);
    g_occupancy_query = nullptr;
    if (!known || occ <= 0) return;
    const int64_t R = 64 / s.lpr;
    int64_t nb = std::min<int64_t>({(int64_t)kMaxNb, (int64_t)occ * h->num_cu, (I + s.waves * R - 1) / (s.waves * R)});
    nb = std::max<int64_t>(1, nb);
    s.rpb = (I + nb - 1) / nb;
    s.nb = (int)((I + s.rpb - 1) / s.rpb);
}

// ---------------------------------------------------------------- helpers --
ot_status copy_in(ot_assoc* h, void* dst, const void* src, size_t bytes, ot_mem mem) {
    HIPCHK(h, hipMemcpyAsync(dst, src, bytes, mem == OT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                             h->stream));
    return OT_OK;
}

ot_status read_vec(ot_assoc* h, const double* p, int64_t n, ot_mem mem, std::vector<double>& out) {
    out.resize((size_t)n);
    if (mem == OT_MEM_HOST) {
        std::memcpy(out.data(), p, sizeof(double) * (size_t)n);
    } else {
        HIPCHK(h, hipMemcpyAsync(out.data(), p, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return OT_OK;
}

double ksum(const std::vector<double>& v) {
    double s = 0.0, c = 0.0;
    for (double x : v) {
        double t = s + x;
        c += (std::fabs(s) >= std::fabs(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    return s + c;
}

ot_status validate_desc(ot_assoc* h, const ot_cost_desc* c) {
    if (!c) return fail(h, OT_EINVAL, "cost descriptor is NULL");
    if (c->I < 1 || c->J < 1 || c->I > h->I_max || c->J > h->J_max)
        return fail(h, OT_EINVAL, "instance %lld x %lld outside 1..%lld x 1..%lld", (long long)c->I, (long long)c->J,
                    (long long)h->I_max, (long long)h->J_max);
    if (c->mem != OT_MEM_HOST && c->mem != OT_MEM_DEVICE) return fail(h, OT_EINVAL, "bad memory space");
    if ((c->kind == OT_COST_DENSE || c->kind == OT_COST_RATES) && c->ld != 0 && c->ld < c->J)
        return fail(h, OT_EINVAL, "row stride ld = %lld is below J = %lld", (long long)c->ld, (long long)c->J);
    switch (c->kind) {
        case OT_COST_DENSE:
        case OT_COST_RATES:
            if (!c->data) return fail(h, OT_EINVAL, "cost data is NULL");
            if (c->dtype != OT_F32 && c->dtype != OT_F64) return fail(h, OT_EINVAL, "bad dtype");
            if (c->kind == OT_COST_RATES && !(c->scale > 0.0 && std::isfinite(c->scale)))
                return fail(h, OT_EINVAL, "rates need a positive finite scale");
            break;
        case OT_COST_GEOMETRY: {
            const ot_geometry& g = c->geom;
            if (!g.dev_xy || !g.rrh_xy) return fail(h, OT_EINVAL, "geometry positions are NULL");
            if (!(g.tx_power_w > 0) || !(g.ref_gain > 0) || !(g.pathloss_exp > 0) || !(g.min_dist_m > 0) ||
                !(g.shadow_sigma_db >= 0) || !(g.noise_w >= 0) || !(g.bandwidth_hz > 0) ||
                !std::isfinite(g.tx_power_w + g.ref_gain + g.pathloss_exp + g.min_dist_m + g.shadow_sigma_db +
                               g.noise_w + g.bandwidth_hz))
                return fail(h, OT_EINVAL, "geometry constants out of range");
            if (!(c->scale > 0.0 && std::isfinite(c->scale)))
                return fail(h, OT_EINVAL, "geometry costs need a positive finite scale");
            break;
        }
        case OT_COST_EUCLID:
            if (!c->geom.dev_xy || !c->geom.rrh_xy) return fail(h, OT_EINVAL, "positions are NULL");
            if (!(c->scale > 0.0 && std::isfinite(c->scale)))
                return fail(h, OT_EINVAL, "distance costs need a positive finite scale");
            break;
        default:
            return fail(h, OT_EINVAL, "unknown cost kind %d", (int)c->kind);
    }
    return OT_OK;
}

ot_status ensure_stage(ot_assoc* h, size_t bytes) {
    if (h->stage_bytes >= bytes) return OT_OK;
    if (!h->ws_owned)  // a caller's workspace: the library allocates nothing
        return fail(h, OT_ENOMEM, "staging a host-memory matrix needs %zu bytes beyond the workspace's fixed "
                                  "buffers (%zu available)", bytes, h->stage_bytes);
    if (h->stage) otk_host::dev_free(h->stage);
    h->stage = nullptr;
    h->stage_bytes = 0;
    HIPCHK(h, otk_host::dev_malloc(&h->stage, bytes));
    h->stage_bytes = bytes;
    return OT_OK;
}


// Brings the cost of `c` onto the device: host matrices are staged, device
// matrices are referenced, positions are copied (and, for the geometry cost,
// its per-device set-up pass runs). Afterwards the handle can rebuild the source without the caller.
// Value checks of the cost: kCheckNone, kCheckNow (the host waits for the
// verdict) or kCheckDeferred (the verdict goes into the control block, bit 8
// of input_bad, and ends the solve on the device).
enum { kCheckNone = 0, kCheckNow = 1, kCheckDeferred = 2 };

ot_status upload_cost(ot_assoc* h, const ot_cost_desc* c, int check) {
    const bool validate_values = check != kCheckNone;
    const bool now = check == kCheckNow;
    int* bad = now ? h->bad : &h->ctl->input_bad;
    const int bit = now ? 1 : 8;
    Ctl* ectl = now ? nullptr : h->ctl;
    const int64_t I = c->I, J = c->J, ld = ld_of(*c), n = I * J;
    h->retained = false;
    h->last = *c;
    if (c->kind != OT_COST_GEOMETRY && c->kind != OT_COST_EUCLID) {
        const size_t esz = c->dtype == OT_F32 ? 4 : 8;
        const void* data = c->data;
        if (c->mem == OT_MEM_HOST) {
            // the padded rows travel whole (I x ld), so the stride is kept
            const size_t bytes = (size_t)(I * ld) * esz;
            ot_status st = ensure_stage(h, bytes);
            if (st) return st;
            HIPCHK(h, hipMemcpyAsync(h->stage, data, bytes, hipMemcpyHostToDevice, h->stream));
            data = h->stage;
        }
        if (validate_values) {
            if (now) HIPCHK(h, hipMemsetAsync(h->bad, 0, sizeof(int), h->stream));
            const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
            const int Ji = (int)J;
            if (c->dtype == OT_F32) {
                if (c->kind == OT_COST_DENSE) hipLaunchKernelGGL((k_validate<float, false>), dim3(grid), dim3(256), 0, h->stream, (const float*)data, I, Ji, ld, bad, bit, ectl);
                else hipLaunchKernelGGL((k_validate<float, true>), dim3(grid), dim3(256), 0, h->stream, (const float*)data, I, Ji, ld, bad, bit, ectl);
            } else {
                if (c->kind == OT_COST_DENSE) hipLaunchKernelGGL((k_validate<double, false>), dim3(grid), dim3(256), 0, h->stream, (const double*)data, I, Ji, ld, bad, bit, ectl);
                else hipLaunchKernelGGL((k_validate<double, true>), dim3(grid), dim3(256), 0, h->stream, (const double*)data, I, Ji, ld, bad, bit, ectl);
            }
            int hbad = 0;
            if (now) {
                HIPCHK(h, hipMemcpyAsync(&hbad, h->bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
                HIPCHK(h, hipStreamSynchronize(h->stream));
            }
            if (hbad)
                return fail(h, OT_EINVAL, c->kind == OT_COST_DENSE ? "cost matrix has non-finite entries"
                                                                  : "rate matrix has entries that are not finite and positive");
        }
        h->cost_dev = data;
        h->retained = true;
        return OT_OK;
    }
    ot_status st = copy_in(h, h->xy_dev, c->geom.dev_xy, sizeof(float) * 2 * (size_t)I, c->mem);
    if (st) return st;
    st = copy_in(h, h->xy_rrh, c->geom.rrh_xy, sizeof(float) * 2 * (size_t)J, c->mem);
    if (st) return st;
    if (validate_values) {
        if (now) HIPCHK(h, hipMemsetAsync(h->bad, 0, sizeof(int), h->stream));
        hipLaunchKernelGGL(k_validate_xy, dim3((unsigned)std::min<int64_t>(1024, (2 * I + 255) / 256)), dim3(256), 0, h->stream, h->xy_dev, 2 * I, bad, bit, ectl);
        hipLaunchKernelGGL(k_validate_xy, dim3((unsigned)std::min<int64_t>(1024, (2 * J + 255) / 256)), dim3(256), 0, h->stream, h->xy_rrh, 2 * J, bad, bit, ectl);
        int hbad = 0;
        if (now) {
            HIPCHK(h, hipMemcpyAsync(&hbad, h->bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
        }
        if (hbad) return fail(h, OT_EINVAL, "geometry positions have non-finite entries");
    }
    if (c->kind == OT_COST_EUCLID) {  // distances need no per-device set-up
        h->cost_dev = nullptr;
        h->retained = true;
        return OT_OK;
    }
    GeoSrc s{};
    s.dev_xy = h->xy_dev;
    s.rrh_xy = h->xy_rrh;
    s.s_all = h->s_all;
    s.s_ex = h->s_ex;
    s.j1 = h->j1;
    s.k = geo_const(c->geom, c->scale);
    const dim3 pg((unsigned)((I + 3) / 4)), pb(256);
    switch (pow2_at_least((int)((J + 63) / 64))) {
        case 1: hipLaunchKernelGGL(k_geo_prepass<1>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
        case 2: hipLaunchKernelGGL(k_geo_prepass<2>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
        case 4: hipLaunchKernelGGL(k_geo_prepass<4>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
        case 8: hipLaunchKernelGGL(k_geo_prepass<8>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
        case 16: hipLaunchKernelGGL(k_geo_prepass<16>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
        default: hipLaunchKernelGGL(k_geo_prepass<32>, pg, pb, 0, h->stream, s, I, (int)J, h->s_all, h->s_ex, h->j1); break;
    }
    HIPCHK(h, hipGetLastError());
    h->cost_dev = nullptr;
    h->retained = true;
    return OT_OK;
}

// Calls fn(src, data) with the source of the retained cost.
template <class F>
ot_status with_retained(ot_assoc* h, F&& fn) {
    const ot_cost_desc& c = h->last;
    const int64_t J = ld_of(c);  // row stride
    if (c.kind == OT_COST_DENSE) {
        if (c.dtype == OT_F32) { DenseSrc<float> s{}; s.C = (const float*)h->cost_dev; s.ld = J; return fn(s, h->cost_dev); }
        DenseSrc<double> s{}; s.C = (const double*)h->cost_dev; s.ld = J; return fn(s, h->cost_dev);
    }
    if (c.kind == OT_COST_RATES) {
        if (c.dtype == OT_F32) { RatesSrc<float> s{}; s.R = (const float*)h->cost_dev; s.ld = J; s.inv_scale = 1.0 / c.scale; return fn(s, h->cost_dev); }
        RatesSrc<double> s{}; s.R = (const double*)h->cost_dev; s.ld = J; s.inv_scale = 1.0 / c.scale; return fn(s, h->cost_dev);
    }
    if (c.kind == OT_COST_EUCLID) {
        EuclidSrc s{};
        s.dev_xy = h->xy_dev;
        s.rrh_xy = h->xy_rrh;
        s.inv_scale = 1.0 / c.scale;
        return fn(s, (const void*)nullptr);
    }
    GeoSrc s{};
    s.dev_xy = h->xy_dev;
    s.rrh_xy = h->xy_rrh;
    s.s_all = h->s_all;
    s.s_ex = h->s_ex;
    s.j1 = h->j1;
    s.k = geo_const(c.geom, c.scale);
    return fn(s, (const void*)nullptr);
}

// --------------------------------------------------------------- iteration --
struct Solver {
    ot_assoc* h;
    int64_t I;
    int J;
    Shape shape;    // fast (FP32-exponential) iterations
    Shape shape64;  // FP64 iterations
    bool graphs;

    // The sweep of iteration k_from + 1: reads iterate k_from (parity
    // k_from & 1), writes f of the other parity and the column partials.
    template <class Src, bool P64>
    ot_status issue_sweep(const Src& src, int k_from) {
        const Shape& sh = P64 ? shape64 : shape;
        const int pin = k_from & 1, pout = pin ^ 1;
        IterArgs A{};
        A.I = I; A.J = J; A.nch = sh.nch; A.rows_per_block = sh.rpb;
        A.a = h->a; A.la = h->la; A.f_in = h->f[pin]; A.f_out = h->f[pout]; A.g_in = h->g[pin];
        A.col_part = h->col_part; A.res_part = h->res_part; A.ctl = h->ctl; A.prm = h->prm;
        if (!launch_iter<Src, P64>(sh, A, src, h->stream))
            return fail(h, OT_EINVAL, "no iteration kernel for vec=%d nch=%d waves=%d rb=%d", sh.vec, sh.nchT, sh.waves, sh.rb);
        return OT_OK;
    }

    // Iteration k_from + 1: the sweep, then the column combine (new g, the
    // residual and the stop decision).
    template <class Src, bool P64>
    ot_status issue_iter(const Src& src, int k_from, int mode, double stall_below) {
        if (ot_status st = issue_sweep<Src, P64>(src, k_from)) return st;
        const Shape& sh = P64 ? shape64 : shape;
        const int pin = k_from & 1, pout = pin ^ 1;
        ColArgs B{};
        B.J = J; B.nb = sh.nb; B.b = h->b; B.g_in = h->g[pin]; B.g_out = h->g[pout];
        B.col_part = h->col_part; B.res_part = h->res_part; B.ctl = h->ctl; B.prm = h->prm;
        B.mode = mode; B.stall_below = stall_below;
        if (!g_prepare_only)
            hipLaunchKernelGGL(k_colsum, dim3((unsigned)((J + kColsPerWg - 1) / kColsPerWg)), dim3(1024), 0, h->stream, B);
        return OT_OK;
    }

    template <class Src, bool P64>
    ot_status issue_chunk(const Src& src, int k0, int n, int mode, double stall_below) {
        for (int q = 0; q < n; ++q) {
            ot_status st = issue_iter<Src, P64>(src, k0 + q, mode, stall_below);
            if (st) return st;
        }
        return OT_OK;
    }

    template <class Src, bool P64>
    ot_status launch_chunk(const Src& src, int k0, int n, int mode, double stall_below) {
        if (!graphs) return issue_chunk<Src, P64>(src, k0, n, mode, stall_below);
        std::string key;
        auto put = [&](const void* p, size_t b) { key.append((const char*)p, b); };
        const Shape& sh = P64 ? shape64 : shape;
        const int tag[10] = {Src::kTag, (int)P64, k0 & 1, n, mode, J, sh.vec, sh.waves, sh.nb, sh.rb};
        put(tag, sizeof tag);
        put(&I, sizeof I);
        put(&sh.rpb, sizeof sh.rpb);
        put(&stall_below, sizeof stall_below);
        put(&src, sizeof src);
        hipGraphExec_t exec = nullptr;
        for (auto& e : h->graphs)
            if (e.key == key) { exec = e.exec; break; }
        if (!exec) {
            g_prepare_only = true;
            ot_status pst = issue_chunk<Src, P64>(src, k0, n, mode, stall_below);
            g_prepare_only = false;
            if (pst) return pst;
            HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            ot_status st = issue_chunk<Src, P64>(src, k0, n, mode, stall_below);
            hipGraph_t graph = nullptr;
            hipError_t e1 = hipStreamEndCapture(h->stream, &graph);
            if (st) { if (graph) hipGraphDestroy(graph); return st; }
            if (e1 != hipSuccess) return fail(h, OT_EDEVICE, "graph capture failed: %s", hipGetErrorString(e1));
            hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e2 != hipSuccess) return fail(h, OT_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e2));
            if ((int)h->graphs.size() >= kGraphCache) {
                hipGraphExecDestroy(h->graphs.front().exec);
                h->graphs.erase(h->graphs.begin());
            }
            h->graphs.push_back(GraphEntry{key, exec});
        }
        HIPCHK(h, hipGraphLaunch(exec, h->stream));
        return OT_OK;
    }

    // (a handle without events, the no-allocation entry point's, waits for
    // the whole stream instead)
    // (ev_stop goes with every copy: when the host has waited for the last
    // one, the solve's device time is known without another round trip)
    ot_status snapshot(int slot) {
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipMemcpyAsync(&h->ctl_h[slot], h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
        if (h->ev_stop) {
            HIPCHK(h, hipEventRecord(h->ev_stop, h->stream));
            h->stop_recorded = true;
        }
        if (h->ev_slot[slot]) HIPCHK(h, hipEventRecord(h->ev_slot[slot], h->stream));
        return OT_OK;
    }
    ot_status wait(int slot) {
        if (h->ev_slot[slot]) HIPCHK(h, hipEventSynchronize(h->ev_slot[slot]));
        else HIPCHK(h, hipStreamSynchronize(h->stream));
        return OT_OK;
    }

    // Runs chunks until the device sets stop (or done). One chunk stays in
    // flight while the host inspects the previous chunk's control block; the
    // extra chunk issued after the stop does nothing on the device.
    template <class Src, bool P64>
    ot_status run_phase(const Src& src, int mode, int chunk, double stall_below, Ctl& state) {
        hipLaunchKernelGGL(k_ctl_resume, dim3(1), dim3(64), 0, h->stream, h->ctl);
        const int k0 = state.iter;  // chunks are even, so every chunk starts on this parity
        int slot = 0;
        ot_status st = launch_chunk<Src, P64>(src, k0, chunk, mode, stall_below);
        if (st || (st = snapshot(slot))) return st;
        for (;;) {
            if ((st = launch_chunk<Src, P64>(src, k0, chunk, mode, stall_below))) return st;
            if ((st = snapshot(slot ^ 1))) return st;
            if ((st = wait(slot))) return st;
            const Ctl& c = h->ctl_h[slot];
            if (c.stop || c.done) {
                if ((st = wait(slot ^ 1))) return st;
                state = h->ctl_h[slot ^ 1];
                return OT_OK;
            }
            slot ^= 1;
        }
    }

    // The exact check of the iterate in buffers k & 1, then one wait. With
    // h->want_loads (and a narrow enough J) the check also sums the RRH
    // loads of the potentials it checks into h->loads; their partials take
    // the second half of the column-partial block, so the grid is capped at
    // half of its rows. A plan buffer named by ot_assoc_set_plan_output is
    // written by the same pass when it holds I x J.
    template <class Src>
    ot_status run_check(const Src& src, int k, Ctl& out) {
        Shape cs = row64(shape64, J);
        const bool fuse = h->want_loads && check_fuses_loads(cs);
        if (fuse && 2 * cs.nb > kMaxNb) {
            cs.rpb = (I + kMaxNb / 2 - 1) / (kMaxNb / 2);
            cs.nb = (int)((I + cs.rpb - 1) / cs.rpb);
        }
        CheckArgs A{};
        A.I = I; A.J = J; A.nch = cs.nch; A.rows_per_block = cs.rpb;
        A.a = h->a; A.f = h->f[k & 1]; A.g = h->g[k & 1];
        A.col_part = h->col_part; A.stat_part = h->stat_part; A.prm = h->prm;
        A.load_part = fuse ? h->col_part + (size_t)cs.nb * (size_t)J : nullptr;
        // (Alg. 2's solves sum the loads; their plans are not asked for)
        A.plan_out = (fuse || (int64_t)I * J > h->plan_cap) ? nullptr : h->plan_out;
        A.plan_f64 = h->plan_dtype == OT_F64 ? 1 : 0;
        h->loads_fresh = h->plan_fresh = false;
        if (!launch_check<Src>(cs, A, src, h->stream)) return fail(h, OT_EINVAL, "no check kernel for this shape");
        CheckColArgs B{};
        const int ncb = (J + kColsPerWg - 1) / kColsPerWg;
        B.J = J; B.nb = cs.nb; B.b = h->b; B.g = h->g[k & 1]; B.col_part = h->col_part; B.cpart = h->cpart;
        B.load_part = A.load_part; B.loads = h->loads;
        hipLaunchKernelGGL(k_check_cols, dim3((unsigned)ncb), dim3(1024), 0, h->stream, B);
        hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(256), 0, h->stream, (const double*)h->stat_part, cs.nb,
                           (const double*)h->cpart, ncb, h->ctl, (const SolveParams*)h->prm);
        h->loads_fresh = fuse;
        h->plan_fresh = A.plan_out != nullptr;
        ot_status st = snapshot(0);
        if (st || (st = wait(0))) return st;
        out = h->ctl_h[0];
        return OT_OK;
    }
};

// ------------------------------------------------------ cooperative phase --
// Shape of the LDS-resident FP32 phase: one workgroup of kPersistWaves waves
// per CU, rows per workgroup a whole number of wave steps; lanes per row and
// cells per lane by J (column q LPR + sub of a row belongs to lane sub).

struct PersistPlan {
    int lpr = 0, cpl = 0, ncl = 0, rpw = 0, nb = 0, Jp = 0;
    size_t lds = 0;
};

template <class Src>
bool persist_plan(const ot_assoc* h, int64_t I, int J, PersistPlan& p) {
    if (!persist_source<Src>() || h->num_cu < 1 || h->lds_max < 1 || I < 1 || !h->xch) return false;
    // cells per lane: the smallest instantiated width that covers the row
    if (J <= 512) {
        p.lpr = 32;
        const int n = (J + 31) / 32;
        p.cpl = n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : n <= 13 ? 13 : 16;
    } else if (J <= kMaxJ) {
        p.lpr = 64;
        p.cpl = J <= 1024 ? 16 : 32;
    } else {
        return false;
    }
    const int slots = kPersistWaves * (64 / p.lpr);  // rows per wave step of the workgroup
    const int64_t per = (int64_t)h->num_cu * slots;
    const int64_t steps = (I + per - 1) / per;
    p.ncl = (J + p.lpr - 1) / p.lpr;
    p.Jp = p.ncl * p.lpr;
    p.rpw = (int)(steps * slots);
    p.nb = (int)((I + p.rpw - 1) / p.rpw);
    p.lds = persist_lds_bytes(p.rpw, J, p.Jp, kPersistWaves, (p.cpl - p.ncl) * p.lpr, p.nb);
    // (a little LDS stays for the kernel's static arrays)
    return p.nb <= h->num_cu && p.nb <= kMaxCoopGroups && p.lds + 2048 <= (size_t)h->lds_max;
}

// Issues the cooperative FP32 phase. `launched` is false (and nothing is
// issued) when the runtime refuses the co-resident grid; the caller then
// runs the chunked launches instead.
template <class Src>
ot_status run_persist(ot_assoc* h, const Src& src, int64_t I, int J, const PersistPlan& p, double stall_below,
                      bool& launched) {
    launched = false;
    const void* kern = persist_kernel<Src>(p.lpr, p.cpl);
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds) != hipSuccess) {
        (void)hipGetLastError();
        return OT_OK;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPersistWaves * 64, p.lds) != hipSuccess ||
        (int64_t)per_cu * h->num_cu < p.nb) {
        (void)hipGetLastError();
        return OT_OK;
    }
    PersistArgs A{};
    A.I = I;
    A.J = J;
    A.Jp = p.Jp;
    A.ncl = p.ncl;
    A.rpw = p.rpw;
    A.max_spin = 1 << 20;  // polls of at least ~1 us each: ~1 s before a wait gives up
    if (g_test_hold > 0) {
        // (test hook, one launch): withhold g at that iteration; waits give up after ~5 ms
        A.hold_iter = g_test_hold;
        A.max_spin = 1 << 12;
        g_test_hold = 0;
    }
    A.stall_below = stall_below;
    A.a = h->a;
    A.b = h->b;
    A.f[0] = h->f[0];
    A.f[1] = h->f[1];
    A.g[0] = h->g[0];
    A.g[1] = h->g[1];
    A.xch = h->xch;
    A.ctl = h->ctl;
    A.prm = h->prm;
    // (the solve's init launch has zeroed the exchange block, unless it
    // could not know that this launch would follow)
    if (!h->xch_zeroed) {
        const size_t nx = persist_exchange_doubles(p.nb, J);
        hipLaunchKernelGGL(k_xch_clear, dim3((unsigned)std::min<size_t>(512, (nx + 255) / 256)), dim3(256), 0,
                           h->stream, h->xch, p.nb, J, h->ctl);
    }
    h->xch_zeroed = false;
    Src sv = src;
    void* args[] = {(void*)&A, (void*)&sv};
    if (h->ev_coop[0]) HIPCHK(h, hipEventRecord(h->ev_coop[0], h->stream));
    const hipError_t e = hipLaunchCooperativeKernel(kern, dim3((unsigned)p.nb), dim3(kPersistWaves * 64), args,
                                                    (unsigned)p.lds, h->stream);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return OT_OK;
    }
    HIPCHK(h, e);
    if (h->ev_coop[1]) HIPCHK(h, hipEventRecord(h->ev_coop[1], h->stream));
    launched = true;
    return OT_OK;
}

// Read-only streaming kernel (the HBM read ceiling of ot_assoc_time_read):
// 16-byte loads, eight in flight per lane, grid-stride. The XOR of the data
// is stored only if it equals a value it practically never takes, so the
// loads are kept and the kernel writes nothing.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
static __global__ __launch_bounds__(256) void k_read_stream(const u32x4* __restrict__ p, size_t n16, uint32_t* sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; q + 7 * stride < n16; q += 8 * stride) {
        u32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(p + q + u * stride);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; q < n16; q += stride) {
        const u32x4 v = __builtin_nontemporal_load(p + q);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u) sink[blockIdx.x & 1023] = acc;
}

// ln a_i of the instance, for the row shifts of the streaming FP32 sweeps.
static __global__ void k_log_a(const double* a, int64_t I, double* la) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I; i += (int64_t)gridDim.x * blockDim.x)
        la[i] = log(a[i]);
}

// Moves iterate (f, g) between buffer pairs in one launch.
static __global__ void k_copy_fg(double* fd, const double* fs, int64_t I, double* gd, const double* gs, int J) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I; i += (int64_t)gridDim.x * blockDim.x)
        fd[i] = fs[i];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < J; j += gridDim.x * blockDim.x) gd[j] = gs[j];
}

// The three phases of a solve. `c` enters with the initial control state and
// leaves with the final one; result_iter names the returned iterate and
// result_par the parity of the buffers that hold it (the iteration's parity,
// except after the cooperative path's check: see there).
template <class Src>
ot_status solve_with(ot_assoc* h, const Src& src, const void* data, int64_t I, int J, double tol, int32_t max_iter,
                     Ctl& c, int& result_iter, int& result_par) {
    const int vec = vec_for<Src>(J, ld_of(h->last), data);
    Solver S{h, I, J, make_shape<Src>(h, I, J, vec, false), make_shape<Src>(h, I, J, vec, true), h->opt.use_graphs != 0};
    fit_grid<Src, false>(h, I, S.shape);
    fit_grid<Src, true>(h, I, S.shape64);
    if (S.shape.nchT > (S.shape.vec == 4 ? 8 : S.shape.vec == 2 ? 16 : 32))
        return fail(h, OT_EINVAL, "J = %d too large for this cost layout", J);
    int chunk = std::max(2, h->opt.chunk);
    chunk += chunk & 1;  // even: every chunk starts on the same buffer parity
    ot_status st;
    const double stall_below = 1e-7;  // FP32 sweeps are not trusted below this
    bool checked = false;
    PersistPlan pp;
    bool persisted = false;
    int coop_par = -1;  // buffers of the iterate the cooperative path checked
    if (h->opt.precision == OT_PREC_FP32 && h->opt.persistent && persist_plan<Src>(h, I, J, pp))
        if ((st = run_persist<Src>(h, src, I, J, pp, stall_below, persisted))) return st;
    h->last_persistent = persisted;
    if (persisted) {
        // polish decided on the device, then the check: one host wait
        const int np = std::max(0, h->opt.polish_iters);
        const unsigned gb = (unsigned)std::min<int64_t>(64, (std::max<int64_t>(I, J) + 255) / 256);
        hipLaunchKernelGGL(k_polish_gate, dim3(gb), dim3(256), 0, h->stream, h->ctl, h->f[0], h->f[1], h->g[0],
                           h->g[1], I, J, tol, stall_below, np);
        if (np > 0 && (st = S.issue_chunk<Src, true>(src, 0, np, kModePolish, 0.0))) return st;
        // the iterate sits in the buffers of parity np & 1 whatever its
        // iteration number (the gate put it there): it is checked and
        // returned from there, and moved to the buffers of its iteration's
        // parity only if more sweeps follow
        if ((st = S.run_check(src, np, c))) return st;
        coop_par = np & 1;
        checked = true;
        h->last_fast_iters = c.iter - c.fp64_iters;  // (the solve starts at iteration 0)
    } else if (h->opt.precision == OT_PREC_FP32) {
        hipLaunchKernelGGL(k_log_a, dim3((unsigned)std::min<int64_t>(1024, (I + 255) / 256)), dim3(256), 0, h->stream,
                           (const double*)h->a, I, h->la);
        if ((st = S.run_phase<Src, false>(src, kModeFast, chunk, stall_below, c))) return st;
        // polish only when the FP32 sweeps stalled short of tol; a residual
        // that met a tol above the FP32 noise threshold goes to the check
        const bool met = c.r_last < c.tol_fast && tol >= stall_below;
        if (!c.done && c.iter < max_iter && !met) {
            const int np = std::max(0, std::min(h->opt.polish_iters, max_iter - c.iter));
            if (np > 0) {
                hipLaunchKernelGGL(k_ctl_resume, dim3(1), dim3(64), 0, h->stream, h->ctl);
                if ((st = S.issue_chunk<Src, true>(src, c.iter, np, kModePolish, 0.0))) return st;
                if ((st = S.snapshot(0)) || (st = S.wait(0))) return st;
                c = h->ctl_h[0];
            }
        }
    }
    if (c.done) {  // inputs rejected, or a numeric failure in the fast phase
        result_iter = c.result_iter;
        result_par = coop_par >= 0 ? coop_par : result_iter & 1;
        h->loads_fresh = h->plan_fresh = false;
        return OT_OK;
    }
    if (!checked && (st = S.run_check<Src>(src, c.iter, c))) return st;
    if (c.done) {  // inputs rejected (seen first by the check of an FP64-precision solve)
        result_iter = c.result_iter;
        result_par = result_iter & 1;
        h->loads_fresh = h->plan_fresh = false;
        return OT_OK;
    }
    result_iter = c.iter;
    result_par = coop_par >= 0 ? coop_par : result_iter & 1;
    if (!(c.chk_violation < tol) && c.iter < max_iter) {
        if (coop_par >= 0 && ((c.iter ^ coop_par) & 1))  // (the FP64 sweeps start from parity c.iter & 1)
            hipLaunchKernelGGL(k_copy_fg, dim3((unsigned)std::min<int64_t>(256, (I + 255) / 256)), dim3(256), 0,
                               h->stream, h->f[c.iter & 1], (const double*)h->f[coop_par], I, h->g[c.iter & 1],
                               (const double*)h->g[coop_par], J);
        if ((st = S.run_phase<Src, true>(src, kModeExact, chunk, 0.0, c))) return st;
        const int k = c.done ? c.result_iter : c.iter;
        const Ctl loop = c;
        if ((st = S.run_check<Src>(src, k, c))) return st;
        c.done = loop.done;
        c.numeric_bad = loop.numeric_bad;
        c.iter = loop.iter;
        c.fp64_iters = loop.fp64_iters;
        result_iter = k;
        result_par = k & 1;
    }
    return OT_OK;
}

// ------------------------------------------------- association quality --
// Workgroups and rows per workgroup of the load passes.
inline void load_grid(const ot_assoc* h, int64_t I, int& nb, int64_t& rpb) {
    const int want = std::max(1, std::min(kMaxNb, 4 * std::max(1, h->num_cu)));
    rpb = std::max<int64_t>(1, (I + want - 1) / want);
    nb = (int)((I + rpb - 1) / rpb);
}

template <class Src, int NCH>
void launch_loads_t(ot_assoc* h, const LoadArgs& A, const Src& src, int nb) {
    auto kern = k_loads<Src, 1, NCH, 8>;
    const size_t ncols = (size_t)NCH * 64;
    const size_t lds = sizeof(double) * std::max((size_t)Src::kStageDoubles * ncols, (size_t)4 * ncols) + 64;
    set_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(512), lds, h->stream, A, src);
}

// One pass of k_loads over the retained cost (load pass when rho is null).
ot_status run_loads(ot_assoc* h, const double* rho, int& nb_out) {
    const int64_t I = h->I;
    const int J = (int)h->J;
    int nb;
    int64_t rpb;
    load_grid(h, I, nb, rpb);
    nb_out = nb;
    LoadArgs A{};
    A.I = I;
    A.J = J;
    A.nch = (J + 63) / 64;
    A.rows_per_block = rpb;
    A.kk = std::log2(std::exp(1.0)) / h->eps;
    A.a = h->a;
    A.f = h->f[h->res_par];
    A.g = h->g[h->res_par];
    A.rho = rho;
    A.col_part = h->col_part;
    A.row_part = h->stat_part;
    ot_status st = with_retained(h, [&](const auto& src, const void*) -> ot_status {
        using S = std::decay_t<decltype(src)>;
        if (J <= 512) launch_loads_t<S, 8>(h, A, src, nb);
        else launch_loads_t<S, 32>(h, A, src, nb);
        return OT_OK;
    });
    if (st) return st;
    HIPCHK(h, hipGetLastError());
    return OT_OK;
}

// load_j (scale 1) or rho_j = kappa load_j and E[N_j] into device buffers.
// When the solve's final check summed the loads (h->loads_valid) they are
// taken from there (one partial row) instead of another pass over the cost.
ot_status device_loads(ot_assoc* h, double scale, double* out_dev, double* en_dev) {
    int nb = 1;
    const double* part = h->loads;
    if (!h->loads_valid) {
        ot_status st = run_loads(h, nullptr, nb);
        if (st) return st;
        part = h->col_part;
    }
    const int J = (int)h->J;
    hipLaunchKernelGGL(k_cols_fin, dim3((unsigned)((J + kFinCols - 1) / kFinCols)), dim3(1024), 0, h->stream,
                       part, nb, J, scale, out_dev, en_dev);
    HIPCHK(h, hipGetLastError());
    return OT_OK;
}

ot_status copy_out(ot_assoc* h, void* dst, const void* src_dev, size_t bytes, ot_mem mem) {
    HIPCHK(h, hipMemcpyAsync(dst, src_dev, bytes, mem == OT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                             h->stream));
    return OT_OK;
}

}  // namespace

// ------------------------------------------- no-allocation solve support --
// ot_assoc_solve_static keeps every device buffer of a solve in this array
// (one copy per GPU, held until the process ends). Its layout is that of a
// handle for kStaticIMax x kStaticJMax instances (ws_layout), about 8.5 MiB.
namespace {
constexpr int64_t kStaticIMax = 32768, kStaticJMax = 512;
constexpr size_t kStaticScratchBytes = (size_t)9 << 20;
constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kStaticMaxDevices] = {};  // the array's device address, per device
thread_local Ctl g_static_ctl[2];             // host mirror of the control block (pageable)
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// =================================================================== C ABI ==
extern "C" {

ot_status ot_assoc_default_options(ot_assoc_options* opt) {
    if (!opt) return OT_EINVAL;
    std::memset(opt, 0, sizeof *opt);
    opt->device = 0;
    opt->stream = nullptr;
    opt->precision = OT_PREC_FP32;
    opt->polish_iters = 1;
    opt->chunk = 8;
    opt->use_graphs = 1;
    opt->batch_tune = 1;
    opt->persistent = 1;
    opt->check_every = 1;
    opt->snapshot_k_split = 1;
    return OT_OK;
}

ot_status ot_assoc_workspace_size(int64_t I_max, int64_t J_max, size_t* bytes) {
    if (!bytes || I_max < 1 || J_max < 1 || J_max > kMaxJ || I_max > ((int64_t)1 << 31)) return OT_EINVAL;
    WsLayout wl;
    ws_layout(I_max, J_max, wl);
    *bytes = wl.total;
    return OT_OK;
}

int64_t ot_assoc_device_allocations(void) { return g_dev_allocs.load(std::memory_order_relaxed); }

const char* ot_assoc_last_error(const ot_assoc* h) { return h ? h->err.c_str() : g_noh_err; }

void ot_assoc_destroy(ot_assoc* h) {
    if (!h) return;
    hipSetDevice(h->device);
    for (auto& e : h->graphs) hipGraphExecDestroy(e.exec);
    if (h->ws && h->ws_owned) otk_host::dev_free(h->ws);
    if (h->stage && !h->stage_in_ws) otk_host::dev_free(h->stage);
    if (h->ctl_h) hipHostFree(h->ctl_h);
    hipEvent_t evs[] = {h->ev_start, h->ev_stop, h->ev_slot[0], h->ev_slot[1], h->ev_coop[0], h->ev_coop[1]};
    for (auto e : evs)
        if (e) hipEventDestroy(e);
    if (h->batch) batch_engine_destroy(h->batch);
    if (h->snap) snap_state_destroy(h->snap);
    if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
    delete h;
}

ot_status ot_assoc_create(ot_assoc** out, int64_t I_max, int64_t J_max, const ot_assoc_options* opt) {
    if (!out) return fail(nullptr, OT_EINVAL, "handle pointer is NULL");
    *out = nullptr;
    if (I_max < 1 || J_max < 1) return fail(nullptr, OT_EINVAL, "I_max and J_max must be >= 1");
    if (J_max > kMaxJ) return fail(nullptr, OT_EINVAL, "J_max %lld exceeds the supported %d RRHs", (long long)J_max, kMaxJ);
    if (I_max > ((int64_t)1 << 31)) return fail(nullptr, OT_EINVAL, "I_max too large");
    ot_assoc_options o;
    ot_assoc_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != OT_PREC_FP32 && o.precision != OT_PREC_FP64) return fail(nullptr, OT_EINVAL, "bad precision");
    if (o.sweep_blocks < 0 || o.sweep_blocks > kMaxNb) return fail(nullptr, OT_EINVAL, "sweep_blocks out of range");
    if (o.chunk < 0 || o.polish_iters < 0) return fail(nullptr, OT_EINVAL, "negative chunk or polish_iters");
    if (o.sweep_rows != 0 && o.sweep_rows != 1 && o.sweep_rows != 2 && o.sweep_rows != 4 && o.sweep_rows != 8)
        return fail(nullptr, OT_EINVAL, "sweep_rows must be 0, 1, 2, 4 or 8");
    if (o.sweep_lanes != 0 && o.sweep_lanes != 16 && o.sweep_lanes != 32 && o.sweep_lanes != 64)
        return fail(nullptr, OT_EINVAL, "sweep_lanes must be 0, 16, 32 or 64");
    if (o.sweep_waves != 0 && o.sweep_waves != 4 && o.sweep_waves != 8)
        return fail(nullptr, OT_EINVAL, "sweep_waves must be 0, 4 or 8");
    if (o.chunk == 0) o.chunk = 8;
    if (o.check_every < 0) return fail(nullptr, OT_EINVAL, "check_every must be >= 0");
    if (o.check_every == 0) o.check_every = 1;
    if (!o.workspace && o.workspace_bytes) return fail(nullptr, OT_EINVAL, "workspace_bytes without a workspace");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, OT_EDEVICE, "no HIP device");
    if (o.device < 0 || o.device >= ndev) return fail(nullptr, OT_EINVAL, "device %d out of range", o.device);
    if (hipSetDevice(o.device) != hipSuccess) return fail(nullptr, OT_EDEVICE, "hipSetDevice failed");
    ot_assoc* h = new ot_assoc();
    h->device = o.device;
    if (hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, o.device) != hipSuccess) h->num_cu = 0;
    if (hipDeviceGetAttribute(&h->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, o.device) != hipSuccess) h->lds_max = 0;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, o.device) != hipSuccess || !coop) h->lds_max = 0;
    h->stream = (hipStream_t)o.stream;
    h->opt = o;
    h->I_max = I_max;
    h->J_max = J_max;
    // every fixed buffer is carved from one device block: the caller's
    // workspace, or one allocation of the same layout
    WsLayout wl;
    ws_layout(I_max, J_max, wl);
    hipError_t e = hipSuccess;
    if (o.workspace) {
        if (o.workspace_bytes < wl.total) {
            fail(nullptr, OT_EINVAL, "workspace of %zu bytes is below the %zu bytes this size needs",
                 o.workspace_bytes, wl.total);
            delete h;
            return OT_EINVAL;
        }
        if ((uintptr_t)o.workspace % kWsAlign != 0) {
            fail(nullptr, OT_EINVAL, "workspace must be %d-byte aligned", kWsAlign);
            delete h;
            return OT_EINVAL;
        }
        h->ws = o.workspace;
        h->ws_owned = false;
        // what lies beyond the fixed buffers stages host-memory matrices
        const size_t tail = o.workspace_bytes - wl.total;
        if (tail > 0) {
            h->stage = (char*)o.workspace + wl.total;
            h->stage_bytes = tail;
            h->stage_in_ws = true;
        }
    } else {
        e = otk_host::dev_malloc(&h->ws, wl.total);
        h->ws_owned = (e == hipSuccess);
    }
    if (e == hipSuccess) carve_ws(h, h->ws, wl);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->ctl_h, 2 * sizeof(Ctl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_stop);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_slot[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_slot[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_coop[0]);
    if (e == hipSuccess) e = hipEventCreate(&h->ev_coop[1]);
    if (e == hipSuccess && !h->stream) {  // graphs cannot be captured on the legacy default stream
        e = hipStreamCreate(&h->stream);
        h->own_stream = (e == hipSuccess);
    }
    if (e != hipSuccess) {
        ot_status st = (e == hipErrorOutOfMemory) ? OT_ENOMEM : OT_EDEVICE;
        fail(nullptr, st, "workspace allocation failed: %s", hipGetErrorString(e));
        ot_assoc_destroy(h);
        return st;
    }
    *out = h;
    return OT_OK;
}

// The body of ot_assoc_solve; also run by ot_assoc_solve_static on a handle
// without events (then the device time is not measured: seconds = 0).
static ot_status solve_impl(ot_assoc* h, const ot_cost_desc* cost, const double* a, const double* b, double eps,
                            double tol, int32_t max_iter, int warm_start, ot_assoc_result* out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    ot_status st = validate_desc(h, cost);
    if (st) return st;
    if (!a || !b) return fail(h, OT_EINVAL, "marginals are NULL");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(h, OT_EINVAL, "eps must be positive and finite");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(h, OT_EINVAL, "tol must be >= 0");
    if (max_iter < 1) return fail(h, OT_EINVAL, "max_iter must be >= 1");
    const int64_t I = cost->I, J = cost->J;
    if (warm_start && !(h->have_pot && h->I == I && h->J == J))
        return fail(h, OT_ESTATE, "warm start needs potentials of a %lld x %lld instance", (long long)I, (long long)J);
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    h->loads_valid = h->loads_fresh = false;
    h->plan_valid = h->plan_fresh = false;
    // marginals, constants and the initial control block are set up and
    // checked on the device (no host round trip before the first sweep)
    const int res_par_prev = h->res_par;
    if (h->ev_start) HIPCHK(h, hipEventRecord(h->ev_start, h->stream));
    const double* a_src = a;
    const double* b_src = b;
    if (cost->mem == OT_MEM_HOST) {
        HIPCHK(h, hipMemcpyAsync(h->a, a, sizeof(double) * I, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->b, b, sizeof(double) * J, hipMemcpyHostToDevice, h->stream));
        a_src = h->a;
        b_src = h->b;
    }
    if (warm_start && res_par_prev != 0) {
        HIPCHK(h, hipMemcpyAsync(h->f[0], h->f[1], sizeof(double) * I, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->g[0], h->g[1], sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream));
    }
    Ctl c{};
    c.has_prev = warm_start ? 1 : 0;
    c.check_every = h->opt.check_every;
    c.last_fp64 = 0;
    c.max_iter = max_iter;
    c.tol = tol;
    c.tol_fast = fast_target(tol, 1e-7);
    c.r_last = __builtin_huge_val();
    for (double& r : c.r_hist) r = __builtin_huge_val();
    InitArgs ia{};
    ia.I = I;
    ia.J = (int)J;
    ia.cold = warm_start ? 0 : 1;
    ia.a_src = a_src;
    ia.b_src = b_src;
    ia.a = h->a;
    ia.b = h->b;
    ia.g0 = h->g[0];
    ia.prm_out = h->prm;
    ia.ctl_out = h->ctl;
    ia.prm = SolveParams{std::log2(std::exp(1.0)) / eps, eps};
    ia.ctl = c;
    // a solve that may take the cooperative FP32 phase has its exchange
    // block zeroed by this launch (nb <= num_cu bounds the launch's layout)
    unsigned init_groups = 1;
    h->xch_zeroed = false;
    h->stop_recorded = false;
    if (h->opt.precision == OT_PREC_FP32 && h->opt.persistent && h->xch && h->num_cu > 0) {
        ia.xch = h->xch;
        ia.nx = (int64_t)persist_exchange_doubles(std::min(h->num_cu, kMaxCoopGroups), (int)J);
        init_groups = 1 + (unsigned)std::min<int64_t>(32, (ia.nx + 4095) / 4096);
        h->xch_zeroed = true;
    }
    hipLaunchKernelGGL(k_solve_init, dim3(init_groups), dim3(1024), 0, h->stream, ia);
    HIPCHK(h, hipGetLastError());

    Ctl fin = c;
    int result_iter = 0, result_par = 0;
    st = upload_cost(h, cost, kCheckDeferred);
    if (!st)
        st = with_retained(h, [&](const auto& src, const void* data) -> ot_status {
            return solve_with(h, src, data, I, (int)J, tol, max_iter, fin, result_iter, result_par);
        });
    if (st) {
        h->solved = h->loads_valid = h->plan_valid = false;
        h->have_pot = false;
        h->retained = false;
        return st;
    }
    float ms = 0.0f;
    h->xch_zeroed = false;
    if (h->ev_start) {
        if (!h->stop_recorded) HIPCHK(h, hipEventRecord(h->ev_stop, h->stream));
        HIPCHK(h, hipEventSynchronize(h->ev_stop));
        hipEventElapsedTime(&ms, h->ev_start, h->ev_stop);
    } else {
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    HIPCHK(h, hipGetLastError());

    if (fin.input_bad) {  // rejected on the device: the handle keeps no result
        h->solved = h->loads_valid = h->plan_valid = false;
        h->have_pot = false;
        h->retained = false;
        const int fb = fin.input_bad;
        if (fb & 1) return fail(h, OT_EINVAL, "device marginal a must be positive and finite");
        if (fb & 2) return fail(h, OT_EINVAL, "RRH marginal b must be positive and finite");
        if (fb & 4)
            return fail(h, OT_EINVAL, "marginals are unbalanced: sum a = %.17g, sum b = %.17g", fin.mass, fin.mass_b);
        if (cost->kind == OT_COST_GEOMETRY || cost->kind == OT_COST_EUCLID)
            return fail(h, OT_EINVAL, "geometry positions have non-finite entries");
        return fail(h, OT_EINVAL, cost->kind == OT_COST_DENSE ? "cost matrix has non-finite entries"
                                                              : "rate matrix has entries that are not finite and positive");
    }
    if (fin.sync_fail) {
        h->solved = h->loads_valid = h->plan_valid = false;
        h->have_pot = false;
        return fail(h, OT_EDEVICE, "a grid barrier of the cooperative FP32 phase gave up waiting");
    }
    h->I = I;
    h->J = J;
    h->eps = eps;
    h->res_par = result_par;
    h->have_pot = true;
    ot_status rs = OT_OK;
    if (fin.numeric_bad || !std::isfinite(fin.chk_violation)) rs = OT_ENUMERIC;
    else if (!(fin.chk_violation < tol)) rs = OT_WARN_MAXITER;
    h->solved = (rs >= 0);
    h->loads_valid = h->solved && h->loads_fresh;
    h->plan_valid = h->solved && h->plan_fresh;
    if (out) {
        out->iterations = result_iter;
        out->fp64_iterations = fin.fp64_iters;
        out->status = rs;
        out->flags = h->last_persistent ? OT_RESULT_PERSISTENT : 0;
        out->marginal_violation = fin.chk_violation;
        out->objective = fin.chk_objective;
        out->reg_objective = fin.chk_reg_objective;
        out->dual_objective = fin.chk_dual;
        out->seconds = ms * 1e-3;
    }
    if (rs == OT_ENUMERIC) return fail(h, OT_ENUMERIC, "non-finite residual or potential during the solve");
    return rs;
}

ot_status ot_assoc_solve(ot_assoc* h, const ot_cost_desc* cost, const double* a, const double* b, double eps,
                         double tol, int32_t max_iter, int warm_start, ot_assoc_result* out) {
    return solve_impl(h, cost, a, b, eps, tol, max_iter, warm_start, out);
}

ot_status ot_assoc_solve_static(int device, void* stream, const float* C, int64_t I, int64_t J, int64_t ld,
                                const double* a, const double* b, double eps, double tol, int32_t max_iter,
                                int warm_start, double* f, double* g, ot_assoc_result* out) {
    if (!C || !a || !b || !f || !g) return fail(nullptr, OT_EINVAL, "a device pointer is NULL");
    if (I < 1 || J < 1 || I > kStaticIMax || J > kStaticJMax)
        return fail(nullptr, OT_EINVAL, "instance %lld x %lld is outside 1..%lld x 1..%lld, the static scratch maximum",
                    (long long)I, (long long)J, (long long)kStaticIMax, (long long)kStaticJMax);
    if (ld != 0 && ld < J) return fail(nullptr, OT_EINVAL, "row stride ld = %lld is below J = %lld", (long long)ld, (long long)J);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, OT_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev || device >= kStaticMaxDevices)
        return fail(nullptr, OT_EINVAL, "device %d out of range", device);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, OT_EDEVICE, "hipSetDevice failed");
    WsLayout wl;
    ws_layout(kStaticIMax, kStaticJMax, wl);
    if (wl.total > kStaticScratchBytes) return fail(nullptr, OT_EDEVICE, "static scratch below its layout");
    // the array's address on this device, looked up once per device with the device current
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (!g_static_ptr[device]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(nullptr, OT_EDEVICE, "hipGetSymbolAddress of the static scratch failed: %s",
                            hipGetErrorString(e));
            g_static_ptr[device] = p;
        }
        base = g_static_ptr[device];
    }
    // a handle on the stack: buffers in the static array, no events, no
    // graphs, the host mirror of the control block in pageable memory
    ot_assoc h;
    ot_assoc_default_options(&h.opt);
    h.opt.device = device;
    h.opt.stream = stream;
    h.opt.use_graphs = 0;
    h.device = device;
    if (hipDeviceGetAttribute(&h.num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) h.num_cu = 0;
    if (hipDeviceGetAttribute(&h.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) h.lds_max = 0;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) h.lds_max = 0;
    h.stream = (hipStream_t)stream;
    h.I_max = kStaticIMax;
    h.J_max = kStaticJMax;
    h.ws = base;
    h.ws_owned = false;
    carve_ws(&h, base, wl);
    h.ctl_h = g_static_ctl;
    h.err_fixed = g_noh_err;
    g_noh_err[0] = 0;
    if (warm_start) {  // the caller's f, g are the starting potentials
        HIPCHK(&h, hipMemcpyAsync(h.f[0], f, sizeof(double) * (size_t)I, hipMemcpyDeviceToDevice, h.stream));
        HIPCHK(&h, hipMemcpyAsync(h.g[0], g, sizeof(double) * (size_t)J, hipMemcpyDeviceToDevice, h.stream));
        h.have_pot = true;
        h.I = I;
        h.J = J;
        h.res_par = 0;
    }
    ot_cost_desc d{};
    d.kind = OT_COST_DENSE;
    d.I = I;
    d.J = J;
    d.mem = OT_MEM_DEVICE;
    d.dtype = OT_F32;
    d.data = C;
    d.ld = ld;
    ot_assoc_result r{};
    const ot_status st = solve_impl(&h, &d, a, b, eps, tol, max_iter, warm_start, &r);
    if (st >= 0) {
        HIPCHK(&h, hipMemcpyAsync(f, h.f[h.res_par], sizeof(double) * (size_t)I, hipMemcpyDeviceToDevice, h.stream));
        HIPCHK(&h, hipMemcpyAsync(g, h.g[h.res_par], sizeof(double) * (size_t)J, hipMemcpyDeviceToDevice, h.stream));
        HIPCHK(&h, hipStreamSynchronize(h.stream));
    }
    if (out && (st >= 0 || st == OT_ENUMERIC)) *out = r;
    return st;
}

ot_status ot_assoc_set_plan_output(ot_assoc* h, void* pi, ot_dtype dtype, int64_t capacity) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (pi && dtype != OT_F32 && dtype != OT_F64) return fail(h, OT_EINVAL, "bad dtype");
    h->plan_out = pi;
    h->plan_dtype = dtype;
    h->plan_cap = pi ? std::max<int64_t>(0, capacity) : 0;
    h->plan_valid = h->plan_fresh = false;
    return OT_OK;
}

ot_status ot_assoc_plan(ot_assoc* h, void* pi, ot_mem mem, ot_dtype dtype) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!h->solved || !h->retained) return fail(h, OT_ESTATE, "no successful solve to take a plan from");
    if (!pi) return fail(h, OT_EINVAL, "plan buffer is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(h, OT_EINVAL, "bad dtype");
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) return fail(h, OT_EINVAL, "bad memory space");
    // written by the solve's final check already (the solve waited for it)
    if (h->plan_valid && mem == OT_MEM_DEVICE && pi == h->plan_out && (int)dtype == h->plan_dtype) return OT_OK;
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = h->I, J = h->J;
    const size_t esz = dtype == OT_F32 ? 4 : 8;
    // device memory: the whole plan in one launch. Host memory: blocks of
    // rows through the handle's work region (nothing is allocated).
    const int64_t block = mem == OT_MEM_DEVICE ? I : std::max<int64_t>(1, (int64_t)(ws_work_bytes(h->I_max, h->J_max) / (esz * (size_t)J)));
    ot_status st = OT_OK;
    for (int64_t r0 = 0; r0 < I && !st; r0 += block) {
        const int64_t r1 = std::min(I, r0 + block);
        void* dst = mem == OT_MEM_DEVICE ? pi : h->work;
        st = with_retained(h, [&](const auto& src, const void* data) -> ot_status {
            using S = std::decay_t<decltype(src)>;
            const Shape s = row64(make_shape<S>(h, I, J, vec_for<S>(J, ld_of(h->last), data)), J);
            const double* f = h->f[h->res_par];
            const double* g = h->g[h->res_par];
            bool ok = dtype == OT_F32 ? launch_plan<S, float>(s, r0, r1, (int)J, f, g, h->prm, (float*)dst, src, h->stream)
                                      : launch_plan<S, double>(s, r0, r1, (int)J, f, g, h->prm, (double*)dst, src, h->stream);
            if (!ok) return fail(h, OT_EINVAL, "no plan kernel for this shape");
            return OT_OK;
        });
        if (!st && mem == OT_MEM_HOST) {
            const size_t bytes = (size_t)((r1 - r0) * J) * esz;
            hipError_t e = hipMemcpyAsync((char*)pi + (size_t)(r0 * J) * esz, h->work, bytes, hipMemcpyDeviceToHost,
                                          h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // the work region is reused by the next block
            if (e != hipSuccess) st = fail(h, OT_EDEVICE, "plan copy failed: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (!st && e != hipSuccess) st = fail(h, OT_EDEVICE, "plan failed: %s", hipGetErrorString(e));
    return st;
}

ot_status ot_assoc_potentials(ot_assoc* h, double* f, double* g, ot_mem mem) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!h->have_pot) return fail(h, OT_ESTATE, "no potentials yet");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const hipMemcpyKind k = mem == OT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (f) HIPCHK(h, hipMemcpyAsync(f, h->f[h->res_par], sizeof(double) * h->I, k, h->stream));
    if (g) HIPCHK(h, hipMemcpyAsync(g, h->g[h->res_par], sizeof(double) * h->J, k, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return OT_OK;
}

ot_status ot_assoc_set_potentials(ot_assoc* h, const double* f, const double* g, int64_t I, int64_t J, ot_mem mem) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!f || !g) return fail(h, OT_EINVAL, "potentials are NULL");
    if (I < 1 || J < 1 || I > h->I_max || J > h->J_max) return fail(h, OT_EINVAL, "sizes out of range");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const hipMemcpyKind k = mem == OT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIPCHK(h, hipMemcpyAsync(h->f[0], f, sizeof(double) * I, k, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->g[0], g, sizeof(double) * J, k, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->I = I;
    h->J = J;
    h->res_par = 0;
    h->have_pot = true;
    h->solved = h->loads_valid = h->plan_valid = false;
    return OT_OK;
}


ot_status ot_assoc_cost_median(ot_assoc* h, const ot_cost_desc* cost, double* median_out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!median_out) return fail(h, OT_EINVAL, "median_out is NULL");
    if (!cost || (cost->kind != OT_COST_RATES && cost->kind != OT_COST_GEOMETRY && cost->kind != OT_COST_EUCLID))
        return fail(h, OT_EINVAL, "the median needs a RATES, GEOMETRY or EUCLID descriptor");
    ot_cost_desc c = *cost;
    c.scale = 1.0;  // C = 1/R
    ot_status st = validate_desc(h, &c);
    if (st) return st;
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = c.I, J = c.J;
    uint64_t rank = (uint64_t)((I * J - 1) / 2);
    uint32_t prefix = 0;
    std::vector<unsigned long long> hh(2048);
    h->solved = h->loads_valid = h->plan_valid = false;  // the handle's retained cost is replaced below
    st = upload_cost(h, &c, kCheckNow);
    if (st) return st;
    st = with_retained(h, [&](const auto& src, const void*) -> ot_status {
        using S = std::decay_t<decltype(src)>;
        const size_t lds = sizeof(double) * S::kStageDoubles * (size_t)J + 8;
        const int grid = (int)std::min<int64_t>(2048, (I + 7) / 8);
        for (int pass = 0; pass < 3; ++pass) {
            HIPCHK(h, hipMemsetAsync(h->hist, 0, sizeof(unsigned long long) * 2048, h->stream));
            hipLaunchKernelGGL(k_median_hist<S>, dim3(grid), dim3(512), lds, h->stream, I, (int)J, pass, prefix, h->hist, src);
            HIPCHK(h, hipMemcpyAsync(hh.data(), h->hist, sizeof(unsigned long long) * 2048, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
            const int nbins = pass == 2 ? 1024 : 2048;
            uint64_t cum = 0;
            int bin = -1;
            for (int q = 0; q < nbins; ++q) {
                if (cum + hh[q] > rank) { bin = q; break; }
                cum += hh[q];
            }
            if (bin < 0) return fail(h, OT_ENUMERIC, "median selection lost its rank (non-finite rates?)");
            rank -= cum;
            prefix = pass == 0 ? (uint32_t)bin : pass == 1 ? ((prefix << 11) | (uint32_t)bin) : ((prefix << 10) | (uint32_t)bin);
        }
        return OT_OK;
    });
    if (st) return st;
    float m;
    std::memcpy(&m, &prefix, sizeof m);
    *median_out = (double)m;
    return OT_OK;
}

ot_status ot_assoc_materialize_cost(ot_assoc* h, const ot_cost_desc* cost, float* C_dev) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!C_dev) return fail(h, OT_EINVAL, "output buffer is NULL");
    if (!cost || (cost->kind != OT_COST_RATES && cost->kind != OT_COST_GEOMETRY && cost->kind != OT_COST_EUCLID))
        return fail(h, OT_EINVAL, "materialisation needs a RATES, GEOMETRY or EUCLID descriptor");
    ot_status st = validate_desc(h, cost);
    if (st) return st;
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = cost->I, J = cost->J;
    h->solved = h->loads_valid = h->plan_valid = false;  // the handle's retained cost is replaced below
    st = upload_cost(h, cost, kCheckNow);
    if (st) return st;
    st = with_retained(h, [&](const auto& src, const void*) -> ot_status {
        using S = std::decay_t<decltype(src)>;
        const size_t lds = sizeof(double) * S::kStageDoubles * (size_t)J + 8;
        const int grid = (int)std::min<int64_t>(4096, (I + 7) / 8);
        hipLaunchKernelGGL(k_materialize<S>, dim3(grid), dim3(512), lds, h->stream, I, (int)J, (int64_t)J, C_dev, src);
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return OT_OK;
    });
    return st;
}

ot_status ot_assoc_fast_phase_time(ot_assoc* h, double* ms, int32_t* iterations) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!ms || !iterations) return fail(h, OT_EINVAL, "output pointer is NULL");
    if (!h->solved || !h->last_persistent)
        return fail(h, OT_ESTATE, "the last solve did not run the cooperative FP32 phase");
    float t = 0.0f;
    HIPCHK(h, hipEventSynchronize(h->ev_coop[1]));
    HIPCHK(h, hipEventElapsedTime(&t, h->ev_coop[0], h->ev_coop[1]));
    *ms = (double)t;
    *iterations = h->last_fast_iters;
    return OT_OK;
}

ot_status ot_assoc_time_sweep(ot_assoc* h, int32_t reps, int fp64, double* ms_per_launch) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!ms_per_launch || reps < 1 || reps > 4096) return fail(h, OT_EINVAL, "reps must be in 1..4096");
    if (!h->solved || !h->retained) return fail(h, OT_ESTATE, "no successful solve to time");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = h->I, J = h->J;
    const int p = h->res_par;
    // the solve's potentials are parked in the work region meanwhile
    double* fs = (double*)h->work;
    double* gs = fs + h->I_max;
    std::vector<hipEvent_t> ev(2, nullptr);
    ot_status st = OT_OK;
    for (auto& x : ev)
        if (hipEventCreate(&x) != hipSuccess) st = fail(h, OT_EDEVICE, "hipEventCreate failed");
    Ctl saved{};
    if (!st) {
        hipMemcpyAsync(fs, h->f[p], sizeof(double) * I, hipMemcpyDeviceToDevice, h->stream);
        hipMemcpyAsync(gs, h->g[p], sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream);
        hipMemcpyAsync(&saved, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
        hipStreamSynchronize(h->stream);
        Ctl c = saved;
        c.stop = 0; c.done = 0; c.has_prev = 1; c.iter = p; c.max_iter = 1 << 30; c.arrive = 0; c.arrive2 = 0;
        c.numeric_bad = 0;
        std::memcpy(&h->ctl_h[0], &c, sizeof c);
        hipMemcpyAsync(h->ctl, &h->ctl_h[0], sizeof(Ctl), hipMemcpyHostToDevice, h->stream);
        // (ln a for the row shifts of the streaming sweeps: a cooperative solve does not compute it)
        hipLaunchKernelGGL(k_log_a, dim3((unsigned)std::min<int64_t>(1024, (I + 255) / 256)), dim3(256), 0, h->stream,
                           (const double*)h->a, I, h->la);
        st = with_retained(h, [&](const auto& src, const void* data) -> ot_status {
            using S = std::decay_t<decltype(src)>;
            const int vec = vec_for<S>(J, ld_of(h->last), data);
            Solver sv{h, I, (int)J, make_shape<S>(h, I, J, vec, false), make_shape<S>(h, I, J, vec, true), false};
            fit_grid<S, false>(h, I, sv.shape);
            fit_grid<S, true>(h, I, sv.shape64);
            // the sweep kernel alone, back to back from alternating parities,
            // between one pair of events: launch gaps included, no event per launch
            HIPCHK(h, hipEventRecord(ev[0], h->stream));
            for (int r = 0; r < reps; ++r) {
                const ot_status s2 = fp64 ? sv.issue_sweep<S, true>(src, p + r) : sv.issue_sweep<S, false>(src, p + r);
                if (s2) return s2;
            }
            HIPCHK(h, hipEventRecord(ev[1], h->stream));
            return OT_OK;
        });
        hipError_t e2 = hipStreamSynchronize(h->stream);
        if (!st && e2 != hipSuccess) st = fail(h, OT_EDEVICE, "timed sweeps failed: %s", hipGetErrorString(e2));
        if (!st) {
            float ms = 0.0f;
            hipEventElapsedTime(&ms, ev[0], ev[1]);
            *ms_per_launch = (double)ms / reps;
        }
        hipMemcpyAsync(h->f[p], fs, sizeof(double) * I, hipMemcpyDeviceToDevice, h->stream);
        hipMemcpyAsync(h->g[p], gs, sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream);
        std::memcpy(&h->ctl_h[0], &saved, sizeof saved);
        hipMemcpyAsync(h->ctl, &h->ctl_h[0], sizeof(Ctl), hipMemcpyHostToDevice, h->stream);
        hipStreamSynchronize(h->stream);
    }
    for (auto& x : ev)
        if (x) hipEventDestroy(x);
    return st;
}


ot_status ot_assoc_test_hold_exchange(int32_t iteration) {
    if (iteration < 0) return OT_EINVAL;
    g_test_hold = iteration;
    return OT_OK;
}

ot_status ot_assoc_time_read(ot_assoc* h, const void* buf, size_t bytes, int32_t reps, double* ms_per_launch) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!buf || !ms_per_launch || bytes < 16 || bytes % 16 != 0 || ((uintptr_t)buf % 16) != 0 || reps < 1 ||
        reps > 4096)
        return fail(h, OT_EINVAL, "time_read needs a 16-byte aligned buffer of a multiple of 16 bytes and reps in 1..4096");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const size_t n16 = bytes / 16;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(1, h->num_cu) * 16,
                                                                            (int64_t)((n16 + 255) / 256)));
    uint32_t* sink = (uint32_t*)h->col_part;  // (written only for an impossible checksum)
    HIPCHK(h, hipEventRecord(h->ev_start, h->stream));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_read_stream, dim3(grid), dim3(256), 0, h->stream, (const u32x4*)buf, n16, sink);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipEventRecord(h->ev_stop, h->stream));
    HIPCHK(h, hipEventSynchronize(h->ev_stop));
    float ms = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop));
    *ms_per_launch = (double)ms / reps;
    return OT_OK;
}

ot_status ot_assoc_rrh_loads(ot_assoc* h, double* loads, ot_mem mem) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!loads) return fail(h, OT_EINVAL, "loads is NULL");
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) return fail(h, OT_EINVAL, "bad memory space");
    if (!h->solved || !h->retained) return fail(h, OT_ESTATE, "no successful solve to take loads from");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    double* out = h->xch;  // (scratch between solves)
    ot_status st = device_loads(h, 1.0, out, nullptr);
    if (!st) st = copy_out(h, loads, out, sizeof(double) * (size_t)h->J, mem);
    if (st) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return OT_OK;
}

ot_status ot_assoc_evaluate(ot_assoc* h, double kappa, double tau, double* rho, double* EN, ot_mem mem,
                            ot_eval_result* out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!out) return fail(h, OT_EINVAL, "out is NULL");
    if (!(kappa > 0.0) || !std::isfinite(kappa) || !(tau > 0.0) || !std::isfinite(tau))
        return fail(h, OT_EINVAL, "kappa and tau must be positive and finite");
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) return fail(h, OT_EINVAL, "bad memory space");
    if (!h->solved || !h->retained) return fail(h, OT_ESTATE, "no successful solve to evaluate");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int J = (int)h->J;
    double* rho_d = h->xch;
    double* en_d = h->xch + J;
    double* tot_d = h->xch + 2 * (size_t)J;
    ot_status st = device_loads(h, kappa, rho_d, en_d);
    if (st) return st;
    int nb = 0;
    if ((st = run_loads(h, rho_d, nb))) return st;
    hipLaunchKernelGGL(k_rows_fin, dim3(1), dim3(256), 0, h->stream, (const double*)h->stat_part, nb, tot_d);
    std::vector<double> hr((size_t)J + 2);
    HIPCHK(h, hipMemcpyAsync(hr.data(), rho_d, sizeof(double) * J, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(hr.data() + J, tot_d, sizeof(double) * 2, hipMemcpyDeviceToHost, h->stream));
    if (rho && (st = copy_out(h, rho, rho_d, sizeof(double) * J, mem))) return st;
    if (EN && (st = copy_out(h, EN, en_d, sizeof(double) * J, mem))) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    ot_eval_result r{};
    r.max_rho = 0.0;
    for (int j = 0; j < J; ++j) {
        r.max_rho = std::max(r.max_rho, hr[j]);
        if (hr[j] >= 1.0) r.overloaded_rrhs += 1;
    }
    r.devices_overloaded = (int32_t)hr[J + 1];
    const bool finite = r.devices_overloaded == 0;
    r.objective = finite ? tau * hr[J] : __builtin_huge_val();
    r.mean_completion = finite ? r.objective / (double)h->I : __builtin_huge_val();
    *out = r;
    return OT_OK;
}

ot_status ot_assoc_maxsinr(ot_assoc* h, const ot_cost_desc* cost, const double* a, int32_t* assoc, double* Lambda) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    ot_status st = validate_desc(h, cost);
    if (st) return st;
    if (!a || !Lambda) return fail(h, OT_EINVAL, "a or Lambda is NULL");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = cost->I;
    const int J = (int)cost->J;
    std::vector<double> ah;
    if ((st = read_vec(h, a, I, cost->mem, ah))) return st;
    for (double v : ah)
        if (!(v >= 0.0) || !std::isfinite(v)) return fail(h, OT_EINVAL, "device traffic a must be non-negative and finite");
    h->solved = h->loads_valid = h->plan_valid = false;  // the handle's retained cost is replaced below
    HIPCHK(h, hipMemcpyAsync(h->a, ah.data(), sizeof(double) * I, hipMemcpyHostToDevice, h->stream));
    if ((st = upload_cost(h, cost, kCheckNow))) return st;
    // rows per workgroup: a multiple of the 64-row chunk, at most kMaxNb workgroups
    int64_t rpb = std::max<int64_t>(kMaxsinrRows, (I + kMaxNb - 1) / kMaxNb);
    rpb = (rpb + kMaxsinrRows - 1) / kMaxsinrRows * kMaxsinrRows;
    const int nb = (int)((I + rpb - 1) / rpb);
    int32_t* assoc_d = nullptr;
    if (assoc && cost->mem == OT_MEM_DEVICE) assoc_d = assoc;
    else if (assoc) assoc_d = (int32_t*)h->work;  // (I_max int32 fit in the work region)
    st = with_retained(h, [&](const auto& src, const void*) -> ot_status {
        using S = std::decay_t<decltype(src)>;
        const size_t lds = sizeof(double) * (size_t)S::kStageDoubles * (size_t)J + 8;
        hipLaunchKernelGGL(k_maxsinr<S>, dim3((unsigned)nb), dim3(256), lds, h->stream, I, J, rpb,
                           (const double*)h->a, src, assoc_d, h->col_part);
        return OT_OK;
    });
    if (!st) {
        double* lam_d = h->xch;
        hipLaunchKernelGGL(k_cols_fin, dim3((unsigned)((J + kFinCols - 1) / kFinCols)), dim3(1024), 0, h->stream,
                           (const double*)h->col_part, nb, J, 1.0, lam_d, (double*)nullptr);
        st = copy_out(h, Lambda, lam_d, sizeof(double) * J, cost->mem);
        if (!st && assoc && assoc_d != assoc)
            st = copy_out(h, assoc, assoc_d, sizeof(int32_t) * (size_t)I, OT_MEM_HOST);
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (st) return st;
    if (e != hipSuccess) return fail(h, OT_EDEVICE, "maxSINR kernels failed: %s", hipGetErrorString(e));
    return OT_OK;
}

ot_status ot_assoc_adaptive(ot_assoc* h, const ot_cost_desc* cost, const double* a, double eps, double tol,
                            int32_t max_iter, double delta, int32_t max_outer, double* q, int32_t* jstar,
                            ot_adaptive_result* out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    ot_status st = validate_desc(h, cost);
    if (st) return st;
    if (!a || !q || !out) return fail(h, OT_EINVAL, "a, q or out is NULL");
    if (max_outer < 1) return fail(h, OT_EINVAL, "max_outer must be >= 1");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, OT_EDEVICE, "hipSetDevice failed");
    const int64_t I = cost->I;
    const int J = (int)cost->J;
    std::vector<double> ah;
    if ((st = read_vec(h, a, I, cost->mem, ah))) return st;
    const double mass = ksum(ah);
    const double d = delta > 0.0 ? delta : 0.01 * mass / J;
    // device copies reused by every solve: a, q, the best potentials; a
    // host-memory matrix is staged once and then referenced
    // (all four in the work region, which holds 2 (I_max + J_max) doubles)
    double* a_d = (double*)h->work;
    double* q_d = a_d + h->I_max;
    double* fb = q_d + h->J_max;
    double* gb = fb + h->I_max;
    auto release = [&]() {};
    // the solves' final checks also sum the RRH loads (J <= 512), so that
    // reading them needs no pass over the cost of its own
    struct WantLoads {
        ot_assoc* h;
        bool prev;
        ~WantLoads() { h->want_loads = prev; }
    } want_guard{h, h->want_loads};
    h->want_loads = true;
    ot_cost_desc dc = *cost;
    auto failed = [&](ot_status s) {
        release();
        return s;
    };
    if (hipMemcpy(a_d, ah.data(), sizeof(double) * I, hipMemcpyHostToDevice) != hipSuccess)
        return failed(fail(h, OT_EDEVICE, "adaptive: copy of a failed"));
    const bool positions = cost->kind == OT_COST_GEOMETRY || cost->kind == OT_COST_EUCLID;
    if (cost->mem == OT_MEM_HOST && !positions) {
        const size_t esz = cost->dtype == OT_F32 ? 4 : 8;
        const size_t bytes = (size_t)(I * ld_of(*cost)) * esz;
        if ((st = ensure_stage(h, bytes))) return failed(st);
        if (hipMemcpy(h->stage, cost->data, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return failed(fail(h, OT_EDEVICE, "adaptive: staging of the cost failed"));
        dc.data = h->stage;
        dc.mem = OT_MEM_DEVICE;
    } else if (cost->mem == OT_MEM_HOST) {
        return failed(fail(h, OT_EINVAL, "adaptive: pass geometry positions in device memory"));
    }
    std::vector<double> qv((size_t)J, mass / J), best_q, loads((size_t)J), best_loads;
    int best = -1, solves = 0, iters = 0;
    double best_max = 0.0, first_max = 0.0;
    ot_assoc_result best_res{};
    for (int k = 0; k < max_outer; ++k) {
        if (hipMemcpy(q_d, qv.data(), sizeof(double) * J, hipMemcpyHostToDevice) != hipSuccess)
            return failed(fail(h, OT_EDEVICE, "adaptive: copy of q failed"));
        ot_assoc_result res{};
        st = ot_assoc_solve(h, &dc, a_d, q_d, eps, tol, max_iter, k > 0 ? 1 : 0, &res);
        if (st < 0) return failed(st);
        ++solves;
        iters += res.iterations;
        if ((st = ot_assoc_rrh_loads(h, loads.data(), OT_MEM_HOST))) return failed(st);
        int js = 0;
        for (int j = 1; j < J; ++j)
            if (loads[j] > loads[js]) js = j;
        const double mx = loads[js];
        if (jstar) jstar[k] = js;
        if (k == 0) first_max = mx;
        if (best >= 0 && !(mx < best_max)) break;
        best = k;
        best_max = mx;
        best_q = qv;
        best_loads = loads;
        best_res = res;
        HIPCHK(h, hipMemcpyAsync(fb, h->f[h->res_par], sizeof(double) * I, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(gb, h->g[h->res_par], sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream));
        if (J < 2 || !(qv[js] - d > 0.0)) break;
        const double step = d / (J - 1);
        std::vector<double> nq((size_t)J);
        for (int j = 0; j < J; ++j) nq[j] = qv[j] + step;
        nq[js] = qv[js] - d;
        qv.swap(nq);
    }
    // the handle holds the best solve's potentials (same instance and eps)
    HIPCHK(h, hipMemcpyAsync(h->f[h->res_par], fb, sizeof(double) * I, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->g[h->res_par], gb, sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream));
    // ... and that solve's loads
    HIPCHK(h, hipMemcpyAsync(h->loads, best_loads.data(), sizeof(double) * J, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->loads_valid = h->solved;
    release();
    std::memcpy(q, best_q.data(), sizeof(double) * J);
    ot_adaptive_result r{};
    r.solves = solves;
    r.best = best;
    r.iterations = iters;
    r.status = best_res.status;
    r.max_load = best_max;
    r.first_max_load = first_max;
    r.delta = d;
    *out = r;
    return (ot_status)best_res.status;
}

}  // extern "C"
