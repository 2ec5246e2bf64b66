// Host runtime of the batched engine and of the request server.
//
// BatchEngine keeps a table of instance slots in device memory, a device
// memory pool that admission draws from (bounded by a byte budget), and two
// generations of work lists that the kernels of batch_kernels.h consume and
// rebuild. A chunk of CHUNK iterations (three persistent launches each) is
// captured once into a HIP graph and replayed for the life of the engine:
// which instances and parts are live is data, not graph structure. The host
// admits new instances between chunks and learns about finished ones from a
// copy of the control blocks taken one chunk behind the device.
//
// ot_assoc_solve_batch admits a whole batch and runs chunks until every
// instance is done. The ot_serve_* entry points admit requests as they
// arrive, as slots and the byte budget allow, while earlier requests are
// still iterating (continuous batching), and keep the potentials of each
// layout resident for warm starts of its next snapshot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ot_assoc.h"
#include "batch_kernels.h"
#include "handle.h"

using namespace otk;

namespace {

constexpr int kChunk = 8;  // iterations per captured chunk (even: list generations alternate)
constexpr int64_t kTailItems = 256;  // at most this many items left: the chunk runs on the tail grids
constexpr double kBatchStallBelow = 1e-7;  // FP32 sweeps are not trusted below this residual
constexpr size_t kAlign = 256;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// ------------------------------------------------------------ device pool --
// First-fit sub-allocator over slabs of device memory, with coalescing of
// neighbouring free blocks inside a slab. Slabs are taken from the device
// only while the total stays within the budget; nothing is returned to the
// device before the pool is destroyed (hipFree would synchronise the device).
class DevicePool {
  public:
    size_t budget = 0;
    size_t reserved = 0;  // bytes of all slabs
    size_t in_use = 0;
    size_t slab_min = (size_t)256 << 20;

    ~DevicePool() { release_all(); }

    void release_all() {
        for (auto& s : slabs_) hipFree(s.base);
        slabs_.clear();
        free_.clear();
        used_.clear();
        reserved = in_use = 0;
    }

    // nullptr when the budget (or the device) cannot provide the bytes
    char* alloc(size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1));
        if (in_use + bytes > budget) return nullptr;
        char* p = take(bytes);
        if (!p) {
            const size_t want = std::max(bytes, slab_min);
            size_t sz = std::min(want, budget - std::min(budget, reserved));
            if (sz < bytes) return nullptr;
            char* base = nullptr;
            if (otk_host::dev_malloc((void**)&base, sz) != hipSuccess) {
                (void)hipGetLastError();
                if (sz > bytes && otk_host::dev_malloc((void**)&base, bytes) == hipSuccess) sz = bytes;
                else { (void)hipGetLastError(); return nullptr; }
            }
            slabs_.push_back({base, sz});
            reserved += sz;
            free_[base] = sz;
            p = take(bytes);
            if (!p) return nullptr;
        }
        used_[p] = bytes;
        in_use += bytes;
        return p;
    }

    void release(char* p) {
        auto it = used_.find(p);
        if (it == used_.end()) return;
        size_t sz = it->second;
        used_.erase(it);
        in_use -= sz;
        const Slab* s = slab_of(p);
        auto nx = free_.lower_bound(p);
        if (nx != free_.end() && nx->first == p + sz && slab_of(nx->first) == s) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == p && slab_of(pv->first) == s) {
                pv->second += sz;
                return;
            }
        }
        free_[p] = sz;
    }

  private:
    struct Slab {
        char* base;
        size_t size;
    };
    std::vector<Slab> slabs_;
    std::map<char*, size_t> free_, used_;

    const Slab* slab_of(char* p) const {
        for (auto& s : slabs_)
            if (p >= s.base && p < s.base + s.size) return &s;
        return nullptr;
    }
    char* take(size_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            char* p = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[p + bytes] = rest;
            return p;
        }
        return nullptr;
    }
};

// One admitted instance, as the host sees it.
struct Slot {
    bool live = false;      // admitted and not yet released
    bool finished = false;  // seen done in a control-block snapshot
    int64_t I = 0;
    int J = 0;
    int64_t ld = 0;
    int parts_cap = 0;
    char* mem = nullptr;  // pool block holding everything below
    BInst d{};
    SolveParams* prm = nullptr;  // for the plan kernel
    double eps = 0.0, mass = 0.0;
    uint64_t ticket = 0, user_tag = 0, layout_key = 0;
    double t_submit = 0.0, t_admit = 0.0;
    long adm_seq = 0;  // snapshots taken before admission (older ones say nothing about it)
    Ctl fin{};
};

}  // namespace

// What one admitted instance needs: its cost, marginals and solve settings,
// plus optional resident potentials to start from.
struct AdmitReq {
    const ot_cost_desc* cost;
    const double* a;
    const double* b;
    double eps, tol;
    int32_t max_iter;
    const double* f0 = nullptr;  // device, warm start (with g0)
    const double* g0 = nullptr;
};

struct BatchEngine {
    int device = 0;
    int num_cu = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    DevicePool pool;
    int cap_slots = 0;
    int cap_items = 0;
    int polish_iters = 1;
    int waves = 8;          // FP32 sweep workgroup size in waves (4 or 8)
    int64_t rpp_rows = 128;  // rows per part
    bool autotune = true;

    // device state
    BInst* tab = nullptr;
    Ctl* ctl = nullptr;
    BList L[2]{};
    char* lists_mem = nullptr;
    // admission staging: one block per admission (jobs, pad jobs, host
    // marginals), pinned on the host and mirrored on the device; two sets
    // used in turn, so an admission waits only for the one before last
    char* blob_h[2] = {nullptr, nullptr};
    char* blob_d[2] = {nullptr, nullptr};
    size_t blob_cap[2] = {0, 0};
    int* relay_h = nullptr;  // relayout: slots and item bases
    int* relay_d = nullptr;
    Ctl* snap[2] = {nullptr, nullptr};
    hipEvent_t ev_snap[2] = {nullptr, nullptr}, ev_adm[2] = {nullptr, nullptr};
    bool adm_pending[2] = {false, false};
    int adm_set = 0;  // staging set of the next admission
    ot_status wait_staging(int set);
    ot_status ensure_blob(int set, size_t bytes);

    std::vector<Slot> slots;
    std::vector<int> free_slots;
    int hi_slot = 0;  // slots [0, hi_slot) may be live
    int n_live_running = 0;
    int64_t items_running = 0;  // parts at the finest layout of admitted, unfinished instances (bounds the lists)
    long seq = 0;               // snapshots taken so far

    // captured chunks, per FP32 workgroup size (wi) and grid set (bulk, or the
    // tail: at most kTailItems items left at the finest layout, launched on
    // smaller grids); index 2 wi + tail
    hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    int graph_polish[4] = {-1, -1, -1, -1};  // polish_iters each graph was captured with
    int grid32[2] = {0, 0}, grid64 = 0, gridc = 0;
    size_t lds32[2] = {0, 0}, lds64 = 0;

    // snapshot pipeline
    long chunks = 0;
    int snap_pending = -1;  // slot of the snapshot in flight, -1 none
    int snap_hi = 0;
    long snap_seq[2] = {0, 0};


    ot_assoc* helper = nullptr;  // materialises geometry costs
    std::vector<int> tab_order;  // slots of the last ot_assoc_solve_batch, in request order

    ~BatchEngine();
    ot_status fail(ot_status st, const char* fmt, ...);
    ot_status init(int dev, hipStream_t st, int slots_cap, int items_cap, size_t budget);
    ot_status prepare_kernels();
    ot_status capture(int widx);
    ot_status admit(const std::vector<AdmitReq>& reqs, std::vector<int>& out_slots, bool strict);
    ot_status upload_cost(Slot& s, const ot_cost_desc* c, char* C_mem, char* stage, PadJob* pad, GeoJob* geo);
    ot_status launch_chunk();
    ot_status collect(bool wait, std::vector<int>& finished);
    ot_status drain_snapshot(std::vector<int>* finished);
    void apply_snapshot(int which, int hi, std::vector<int>* finished);
    void release(int slot);
    ot_status tune(const std::vector<int>& batch_slots);
    std::string tune_key(const std::vector<int>& batch_slots) const;
    ot_status relayout(const std::vector<int>& batch_slots, int w, int64_t rpp);
    int widx() const { return waves == 4 ? 0 : 1; }
    int gidx() const { return 2 * widx() + (items_running <= kTailItems ? 1 : 0); }
};

#define ECHK(e, call)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess)                                                                                  \
            return (e)->fail((e_ == hipErrorOutOfMemory) ? OT_ENOMEM : OT_EDEVICE, "%s failed: %s (%s:%d)", #call, \
                             hipGetErrorString(e_), __FILE__, __LINE__);                                        \
    } while (0)

ot_status BatchEngine::fail(ot_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return st;
}

BatchEngine::~BatchEngine() {
    hipSetDevice(device);
    if (stream) hipStreamSynchronize(stream);
    for (auto g : graph)
        if (g) hipGraphExecDestroy(g);
    void* dev_bufs[] = {tab, ctl, lists_mem, blob_d[0], blob_d[1], relay_d};
    for (void* p : dev_bufs)
        if (p) hipFree(p);
    void* host_bufs[] = {snap[0], snap[1], blob_h[0], blob_h[1], relay_h};
    for (void* p : host_bufs)
        if (p) hipHostFree(p);
    hipEvent_t evs[] = {ev_snap[0], ev_snap[1], ev_adm[0], ev_adm[1]};
    for (auto e : evs)
        if (e) hipEventDestroy(e);
    if (helper) ot_assoc_destroy(helper);
    pool.release_all();
    if (own_stream && stream) hipStreamDestroy(stream);
}

void batch_engine_destroy(BatchEngine* e) { delete e; }

ot_status BatchEngine::init(int dev, hipStream_t st, int slots_cap, int items_cap, size_t budget) {
    device = dev;
    ECHK(this, hipSetDevice(dev));
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || num_cu <= 0)
        return fail(OT_EDEVICE, "cannot query the number of compute units");
    if (st) {
        stream = st;
    } else {
        ECHK(this, hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        own_stream = true;
    }
    cap_slots = slots_cap;
    cap_items = items_cap;
    pool.budget = budget;
    ECHK(this, otk_host::dev_malloc((void**)&tab, sizeof(BInst) * cap_slots));
    ECHK(this, otk_host::dev_malloc((void**)&ctl, sizeof(Ctl) * cap_slots));
    const size_t item_bytes = align_up(sizeof(BItem) * (size_t)cap_items);
    const size_t inst_bytes = align_up(sizeof(int) * (size_t)cap_slots);
    const size_t gen_bytes = 2 * item_bytes + inst_bytes + kAlign;
    ECHK(this, otk_host::dev_malloc((void**)&lists_mem, 2 * gen_bytes));
    for (int g = 0; g < 2; ++g) {
        char* p = lists_mem + g * gen_bytes;
        L[g].it32 = (BItem*)p;
        L[g].it64 = (BItem*)(p + item_bytes);
        L[g].inst = (int*)(p + 2 * item_bytes);
        L[g].cnt = (int*)(p + 2 * item_bytes + inst_bytes);
    }
    ECHK(this, hipMemsetAsync(lists_mem, 0, 2 * gen_bytes, stream));
    for (int q = 0; q < 2; ++q) ECHK(this, hipEventCreateWithFlags(&ev_adm[q], hipEventDisableTiming));
    ECHK(this, hipHostMalloc(&relay_h, sizeof(int) * 2 * cap_slots));
    ECHK(this, otk_host::dev_malloc((void**)&relay_d, sizeof(int) * 2 * cap_slots));
    for (auto& s : snap) ECHK(this, hipHostMalloc(&s, sizeof(Ctl) * cap_slots));
    for (auto& e : ev_snap) ECHK(this, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    slots.assign(cap_slots, Slot{});
    free_slots.clear();
    for (int q = cap_slots - 1; q >= 0; --q) free_slots.push_back(q);
    ECHK(this, hipStreamSynchronize(stream));
    return prepare_kernels();
}

// LDS of the batch sweeps: the largest column class (32 lanes x 4 chunks x 4)
// staged as FP64 + FP32 g, or reused by the workgroup reduction.
static size_t bsweep_lds(bool p64, int w) {
    const size_t ncols = 512;
    const size_t a = sizeof(double) * (ncols + ncols / 2);
    const size_t red = (p64 ? 8 : 4) * (size_t)w * 4 * 256;  // LPR 16: R = 4 rows, up to 256 columns
    const size_t red32 = (p64 ? 8 : 4) * (size_t)w * 2 * 512;  // LPR 32: R = 2 rows, 512 columns
    const size_t chk = sizeof(double) * (size_t)(w / 2) * 2 * 64 * 4;
    return std::max({a, red, red32, chk});
}

template <class K>
static int occupancy(K kern, int threads, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, lds) != hipSuccess) n = 0;
    return n;
}

ot_status BatchEngine::prepare_kernels() {
    lds32[0] = bsweep_lds(false, 4);
    lds32[1] = bsweep_lds(false, 8);
    lds64 = bsweep_lds(true, 8);
    const int o4 = occupancy(k_bsweep<false, 4>, 256, lds32[0]);
    const int o8 = occupancy(k_bsweep<false, 8>, 512, lds32[1]);
    const int o64 = occupancy(k_bsweep<true, 8>, 512, lds64);
    const int oc = occupancy(k_bcombine, 1024, 0);
    if (o4 <= 0 || o8 <= 0 || o64 <= 0 || oc <= 0) return fail(OT_EDEVICE, "batch kernels do not fit on a CU");
    grid32[0] = o4 * num_cu;
    grid32[1] = o8 * num_cu;
    grid64 = o64 * num_cu;
    gridc = oc * num_cu;
    return OT_OK;
}

ot_status BatchEngine::capture(int gi) {
    if (graph[gi] && graph_polish[gi] == polish_iters) return OT_OK;
    if (graph[gi]) {
        hipGraphExecDestroy(graph[gi]);
        graph[gi] = nullptr;
    }
    const int wi = gi >> 1;
    const bool tail = (gi & 1) != 0;
    // (grid sizes only change which workgroup takes which item: results are
    // the same on either grid set)
    const int g32 = tail ? std::min(grid32[wi], num_cu) : grid32[wi];
    const int g64 = tail ? std::min(grid64, 64) : grid64;
    const int gc = tail ? std::min(gridc, 32) : gridc;
    BParams P{polish_iters, kBatchStallBelow};
    hipGraph_t g = nullptr;
    ECHK(this, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < kChunk; ++t) {
        const BList& in = L[t & 1];
        const BList& out = L[(t + 1) & 1];
        const BInst* T = tab;
        if (wi == 0)
            hipLaunchKernelGGL((k_bsweep<false, 4>), dim3(g32), dim3(256), lds32[0], stream, T,
                               (const BItem*)in.it32, (const int*)in.cnt, out.cnt);
        else
            hipLaunchKernelGGL((k_bsweep<false, 8>), dim3(g32), dim3(512), lds32[1], stream, T,
                               (const BItem*)in.it32, (const int*)in.cnt, out.cnt);
        hipLaunchKernelGGL((k_bsweep<true, 8>), dim3(g64), dim3(512), lds64, stream, T, (const BItem*)in.it64,
                           (const int*)in.cnt, out.cnt);
        hipLaunchKernelGGL(k_bcombine, dim3(gc), dim3(1024), 0, stream, tab, in, out, P);
    }
    hipError_t e1 = hipStreamEndCapture(stream, &g);
    if (e1 != hipSuccess) return fail(OT_EDEVICE, "graph capture failed: %s", hipGetErrorString(e1));
    graph_polish[gi] = polish_iters;
    hipError_t e2 = hipGraphInstantiate(&graph[gi], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(OT_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e2));
    return OT_OK;
}

// Bytes of one instance's block: cost (unless referenced), marginals,
// potentials (two parities), parts partials, solve constants.
static size_t slot_bytes(int64_t I, int J, int64_t ld, int parts_cap, bool own_cost) {
    size_t b = 0;
    if (own_cost) b += align_up(sizeof(float) * (size_t)I * ld);
    b += align_up(sizeof(double) * I) + align_up(sizeof(double) * J);                      // a, b
    b += 2 * align_up(sizeof(double) * I) + 2 * align_up(sizeof(double) * J);              // f, g
    b += align_up(sizeof(double) * (size_t)parts_cap * J) + align_up(sizeof(double) * parts_cap);  // col, res
    b += align_up(sizeof(double) * (size_t)parts_cap * 5) + align_up(sizeof(SolveParams));
    return b;
}

static int64_t parts_of(int64_t I, int64_t rpp) { return (I + rpp - 1) / rpp; }

// Costs regenerated from positions (geometry, distances): device memory only,
// materialised into the slot's padded FP32 matrix at admission.
static bool from_positions(const ot_cost_desc* c) {
    return c->kind == OT_COST_GEOMETRY || c->kind == OT_COST_EUCLID;
}

ot_status BatchEngine::upload_cost(Slot& s, const ot_cost_desc* c, char* C_mem, char* stage, PadJob* pad,
                                   GeoJob* geo) {
    const int64_t I = s.I;
    const int J = s.J;
    const int64_t ld = s.ld;
    float* dst = (float*)C_mem;
    pad->src = nullptr;
    geo->dst = nullptr;
    if (from_positions(c)) {
        double scale = c->scale;
        if (!(scale > 0.0)) {
            // the median of 1/R needs host read-backs: a handle of the
            // single-instance path on this engine's stream computes it
            if (!helper || helper->I_max < I) {
                if (helper) ot_assoc_destroy(helper);
                helper = nullptr;
                ot_assoc_options o;
                ot_assoc_default_options(&o);
                o.device = device;
                o.stream = stream;
                ot_status st = ot_assoc_create(&helper, std::max<int64_t>(I, 1 << 15), kBatchMaxJ, &o);
                if (st) return fail(st, "helper handle: %s", ot_assoc_last_error(nullptr));
            }
            ot_status st = ot_assoc_cost_median(helper, c, &scale);
            if (st) return fail(st, "cost median: %s", ot_assoc_last_error(helper));
        }
        // a job of the admission's two set-up launches: per-device
        // interference sums (geometry, into the staging block), then the
        // padded FP32 matrix; non-finite positions surface as a numeric
        // failure of the solve
        *geo = GeoJob{};
        geo->dst = dst;
        geo->I = I;
        geo->ld = ld;
        geo->J = J;
        if (c->kind == OT_COST_EUCLID) {
            geo->kind = 1;
            geo->dist.dev_xy = (const float*)c->geom.dev_xy;
            geo->dist.rrh_xy = (const float*)c->geom.rrh_xy;
            geo->dist.inv_scale = 1.0 / scale;
            return OT_OK;
        }
        geo->kind = 0;
        GeoSrc& g = geo->geo;
        g.dev_xy = (const float*)c->geom.dev_xy;
        g.rrh_xy = (const float*)c->geom.rrh_xy;
        geo->s_all = (double*)stage;
        geo->s_ex = geo->s_all + I;
        geo->j1 = (int*)(geo->s_ex + I);
        g.s_all = geo->s_all;
        g.s_ex = geo->s_ex;
        g.j1 = geo->j1;
        g.k = geo_const(c->geom, scale);
        return OT_OK;
    }
    // dense or rate matrices: a padded-copy job, run for the whole admission
    const size_t esz = c->dtype == OT_F32 ? 4 : 8;
    const int64_t lds = c->ld ? c->ld : J;
    const void* src = c->data;
    if (c->mem == OT_MEM_HOST) {
        ECHK(this, hipMemcpyAsync(stage, c->data, esz * (size_t)(I * lds), hipMemcpyHostToDevice, stream));
        src = stage;
    }
    pad->src = src;
    pad->dst = dst;
    pad->I = I;
    pad->lds = lds;
    pad->ld = ld;
    pad->inv_scale = c->kind == OT_COST_RATES ? 1.0 / c->scale : 1.0;
    pad->J = J;
    pad->kind = c->kind == OT_COST_RATES ? 1 : 0;
    pad->f64 = c->dtype == OT_F64 ? 1 : 0;
    return OT_OK;
}


static ot_status check_desc(BatchEngine* e, const ot_cost_desc* c) {
    if (!c) return e->fail(OT_EINVAL, "cost descriptor is NULL");
    if (c->I < 1 || c->J < 1 || c->J > kBatchMaxJ || c->I > ((int64_t)1 << 26))
        return e->fail(OT_EINVAL, "batched instance %lld x %lld outside 1..2^26 x 1..%d", (long long)c->I,
                       (long long)c->J, kBatchMaxJ);
    if (c->mem != OT_MEM_HOST && c->mem != OT_MEM_DEVICE) return e->fail(OT_EINVAL, "bad memory space");
    switch (c->kind) {
        case OT_COST_DENSE:
        case OT_COST_RATES:
            if (!c->data) return e->fail(OT_EINVAL, "cost matrix is NULL");
            if (c->dtype != OT_F32 && c->dtype != OT_F64) return e->fail(OT_EINVAL, "bad dtype");
            if (c->kind == OT_COST_RATES && !(c->scale > 0.0 && std::isfinite(c->scale)))
                return e->fail(OT_EINVAL, "rates need scale > 0");
            if (c->ld != 0 && c->ld < c->J) return e->fail(OT_EINVAL, "row stride below J");
            break;
        case OT_COST_GEOMETRY:
        case OT_COST_EUCLID:
            if (c->mem != OT_MEM_DEVICE) return e->fail(OT_EINVAL, "batched positions must be in device memory");
            if (!c->geom.dev_xy || !c->geom.rrh_xy) return e->fail(OT_EINVAL, "positions are NULL");
            if (std::isinf(c->scale)) return e->fail(OT_EINVAL, "scale must be finite (<= 0: the median)");
            break;
        default:
            return e->fail(OT_EINVAL, "unknown cost kind");
    }
    return OT_OK;
}

// Admits the requests in order. strict: every request must fit now (else
// OT_ENOMEM and nothing is admitted); otherwise admits the longest prefix
// that fits and reports the admitted slots. Settings are checked here,
// marginal values on the device, so admission never waits on the GPU beyond
// the staging set of the admission before last.
ot_status BatchEngine::admit(const std::vector<AdmitReq>& reqs, std::vector<int>& out_slots, bool strict) {
    out_slots.clear();
    if (reqs.empty()) return OT_OK;
    ECHK(this, hipSetDevice(device));
    for (size_t q = 0; q < reqs.size(); ++q) {
        const AdmitReq& r = reqs[q];
        if (ot_status st = check_desc(this, r.cost)) return st;
        if (!r.a || !r.b) return fail(OT_EINVAL, "marginals are NULL");
        if (!(r.eps > 0.0) || !std::isfinite(r.eps)) return fail(OT_EINVAL, "eps must be positive and finite");
        if (!(r.tol >= 0.0) || !std::isfinite(r.tol)) return fail(OT_EINVAL, "tol must be >= 0");
        if (r.max_iter < 1) return fail(OT_EINVAL, "max_iter must be >= 1");
    }
    const int set = adm_set;
    if (ot_status st = wait_staging(set)) return st;
    // staging block: [AdmJob x n][PadJob x n][GeoJob x n][host marginals]
    const size_t n = reqs.size();
    const size_t jobs_b = align_up(sizeof(AdmJob) * n), pads_b = align_up(sizeof(PadJob) * n);
    const size_t geos_b = align_up(sizeof(GeoJob) * n);
    size_t marg_b = 0;
    for (auto& r : reqs)
        if (!from_positions(r.cost) && r.cost->mem == OT_MEM_HOST)
            marg_b += align_up(sizeof(double) * r.cost->I) + align_up(sizeof(double) * r.cost->J);
    if (ot_status st = ensure_blob(set, jobs_b + pads_b + geos_b + marg_b)) return st;
    AdmJob* jobs_h = (AdmJob*)blob_h[set];
    PadJob* pads_h = (PadJob*)(blob_h[set] + jobs_b);
    GeoJob* geos_h = (GeoJob*)(blob_h[set] + jobs_b + pads_b);
    char* marg_h = blob_h[set] + jobs_b + pads_b + geos_b;
    char* marg_d = blob_d[set] + jobs_b + pads_b + geos_b;
    int n_items = 0, n_insts = 0, n_pads = 0, n_geos = 0;
    int64_t n_cap = 0;  // items of this admission at the finest layout
    int64_t pad_rows = 0;  // rows of the largest padded copy
    std::vector<char*> stages;
    auto undo = [&]() {
        for (char* x : stages) pool.release(x);
        for (int k : out_slots) {
            slots[k].finished = true;  // never counted as running
            release(k);
        }
        out_slots.clear();
    };
    const int64_t rpp = rpp_rows;
    for (size_t q = 0; q < n; ++q) {
        const AdmitReq& r = reqs[q];
        const ot_cost_desc* c = r.cost;
        const int64_t I = c->I;
        const int J = (int)c->J;
        // the finest layout: the tuner's smallest rows per part and the layout of
        // instances still running after kFineIter iterations (item counts and
        // the partial buffers are bounded by it)
        const int parts_cap = (int)parts_of(I, kFineRows);
        const int parts = (int)parts_of(I, rpp);
        const int64_t lds = c->ld ? c->ld : J;
        const bool ref = c->kind == OT_COST_DENSE && c->mem == OT_MEM_DEVICE && c->dtype == OT_F32 && J % 4 == 0 &&
                         lds % 4 == 0 && ((uintptr_t)c->data % 16) == 0;
        const int64_t ld = ref ? lds : (J + 3) / 4 * 4;
        if (free_slots.empty() || items_running + n_cap + parts_cap > cap_items) {
            if (strict) {
                undo();
                return fail(OT_ENOMEM, "batch exceeds %d slots / %d work items", cap_slots, cap_items);
            }
            break;
        }
        // staging for host cost matrices and for the geometry set-up pass;
        // released once the work reading it is queued (stream order)
        const size_t esz = c->dtype == OT_F64 ? 8 : 4;
        size_t stage_b = 0;
        if (!ref && !from_positions(c) && c->mem == OT_MEM_HOST) stage_b = esz * (size_t)(I * lds);
        if (c->kind == OT_COST_GEOMETRY) stage_b = (2 * sizeof(double) + sizeof(int)) * (size_t)I;
        char* stage = stage_b ? pool.alloc(stage_b) : nullptr;
        char* mem = (stage_b && !stage) ? nullptr : pool.alloc(slot_bytes(I, J, ld, parts_cap, !ref));
        if (!mem) {
            if (stage) pool.release(stage);
            if (strict) {
                undo();
                return fail(OT_ENOMEM, "batch exceeds the device memory budget (%.3g GB)", pool.budget / 1e9);
            }
            break;
        }
        if (stage) stages.push_back(stage);
        const int k = free_slots.back();
        free_slots.pop_back();
        hi_slot = std::max(hi_slot, k + 1);
        Slot& sl = slots[k];
        sl = Slot{};
        sl.live = true;
        sl.I = I;
        sl.J = J;
        sl.ld = ld;
        sl.parts_cap = parts_cap;
        sl.mem = mem;
        sl.eps = r.eps;
        char* p = mem;
        auto carve = [&](size_t bytes) {
            char* x = p;
            p += align_up(bytes);
            return x;
        };
        BInst& d = sl.d;
        char* C_mem = ref ? nullptr : carve(sizeof(float) * (size_t)I * ld);
        d.C = ref ? (const float*)c->data : (const float*)C_mem;
        d.ld = ld;
        d.I = I;
        d.J = J;
        d.cls = batch_class(J);
        d.nch = (J + batch_class_lpr(d.cls) * 4 - 1) / (batch_class_lpr(d.cls) * 4);
        d.nchk = (J + 255) / 256;
        d.parts = parts;
        d.rpp = rpp;
        d.a = (double*)carve(sizeof(double) * I);
        d.b = (double*)carve(sizeof(double) * J);
        d.f[0] = (double*)carve(sizeof(double) * I);
        d.f[1] = (double*)carve(sizeof(double) * I);
        d.g[0] = (double*)carve(sizeof(double) * J);
        d.g[1] = (double*)carve(sizeof(double) * J);
        d.col_part = (double*)carve(sizeof(double) * (size_t)parts_cap * J);
        d.res_part = (double*)carve(sizeof(double) * parts_cap);
        d.stat_part = (double*)carve(sizeof(double) * (size_t)parts_cap * 5);
        sl.prm = (SolveParams*)carve(sizeof(SolveParams));
        d.prm = sl.prm;
        d.ctl = ctl + k;
        d.kk = std::log2(std::exp(1.0)) / r.eps;
        d.eps = r.eps;
        out_slots.push_back(k);
        if (!ref) {
            PadJob pj{};
            GeoJob gj{};
            ot_status st = upload_cost(sl, c, C_mem, stage, &pj, &gj);
            if (st) {
                undo();
                return st;
            }
            if (pj.src) {
                pads_h[n_pads++] = pj;
                pad_rows = std::max(pad_rows, pj.I);
            }
            if (gj.dst) geos_h[n_geos++] = gj;
        }
        AdmJob& J1 = jobs_h[n_insts];
        J1 = AdmJob{};
        J1.d = d;
        J1.sp = SolveParams{d.kk, d.eps};
        J1.prm_dst = sl.prm;
        if (!from_positions(c) && c->mem == OT_MEM_HOST) {
            std::memcpy(marg_h, r.a, sizeof(double) * I);
            J1.a_src = (const double*)marg_d;
            marg_h += align_up(sizeof(double) * I);
            marg_d += align_up(sizeof(double) * I);
            std::memcpy(marg_h, r.b, sizeof(double) * J);
            J1.b_src = (const double*)marg_d;
            marg_h += align_up(sizeof(double) * J);
            marg_d += align_up(sizeof(double) * J);
        } else {
            J1.a_src = r.a;
            J1.b_src = r.b;
        }
        const bool warm = r.f0 && r.g0;
        J1.f0 = warm ? r.f0 : nullptr;
        J1.g0 = warm ? r.g0 : nullptr;
        Ctl& ci = J1.ci;
        ci.has_prev = warm ? 1 : 0;
        ci.max_iter = r.max_iter;
        ci.tol = r.tol;
        // (no margin here: a batched instance whose check misses tol continues
        // with FP64 sweeps on the device, which costs less than the longer
        // FP32 tail a margin would add to the whole batch)
        ci.tol_fast = r.tol;
        ci.r_last = __builtin_huge_val();
        for (double& x : ci.r_hist) x = __builtin_huge_val();
        ci.phase = kPhFast;
        sl.fin = ci;
        J1.slot = k;
        J1.item_base = n_items;
        J1.inst_pos = n_insts;
        n_items += parts;
        n_cap += parts_cap;
        ++n_insts;
        sl.t_admit = now_s();
        sl.adm_seq = seq;
    }
    // block ranges of the set-up launches
    int pre_blocks = 0, mat_blocks = 0;
    for (int q = 0; q < n_geos; ++q) {
        GeoJob& g = geos_h[q];
        g.pre_blk0 = pre_blocks;
        g.pre_nblk = g.kind == 0 ? (int)((g.I + kGeoJobRowsPre - 1) / kGeoJobRowsPre) : 0;
        g.mat_blk0 = mat_blocks;
        g.mat_nblk = (int)((g.I + kGeoJobRowsMat - 1) / kGeoJobRowsMat);
        pre_blocks += g.pre_nblk;
        mat_blocks += g.mat_nblk;
    }
    if (n_insts) {
        const size_t used = (size_t)(marg_h - blob_h[set]);
        ECHK(this, hipMemcpyAsync(blob_d[set], blob_h[set], used, hipMemcpyHostToDevice, stream));
        if (n_pads)
            hipLaunchKernelGGL(k_bpad_jobs,
                               dim3((unsigned)std::min<int64_t>(256, (pad_rows + kPadRowsPerBlock - 1) / kPadRowsPerBlock),
                                    n_pads),
                               dim3(256), 0, stream, (const PadJob*)(blob_d[set] + jobs_b));
        const GeoJob* geos_d = (const GeoJob*)(blob_d[set] + jobs_b + pads_b);
        if (pre_blocks)
            hipLaunchKernelGGL(k_bgeo_prepass_jobs, dim3(pre_blocks), dim3(256), 0, stream, geos_d, n_geos);
        if (mat_blocks)
            hipLaunchKernelGGL(k_bmat_jobs, dim3(mat_blocks), dim3(512), 0, stream, geos_d, n_geos);
        hipLaunchKernelGGL(k_badmit_jobs, dim3(n_insts), dim3(256), 0, stream, (const AdmJob*)blob_d[set], tab, ctl,
                           L[0]);
        hipLaunchKernelGGL(k_bcount, dim3(1), dim3(64), 0, stream, L[0], n_items, n_insts);
        ECHK(this, hipGetLastError());
        ECHK(this, hipEventRecord(ev_adm[set], stream));
        adm_pending[set] = true;
        adm_set ^= 1;
        n_live_running += n_insts;
        items_running += n_cap;
    }
    for (char* x : stages) pool.release(x);
    return OT_OK;
}

ot_status BatchEngine::ensure_blob(int set, size_t bytes) {
    if (blob_cap[set] >= bytes) return OT_OK;
    if (blob_h[set]) hipHostFree(blob_h[set]);
    if (blob_d[set]) hipFree(blob_d[set]);
    blob_h[set] = blob_d[set] = nullptr;
    blob_cap[set] = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 20);
    ECHK(this, hipHostMalloc(&blob_h[set], cap));
    ECHK(this, otk_host::dev_malloc((void**)&blob_d[set], cap));
    blob_cap[set] = cap;
    return OT_OK;
}

ot_status BatchEngine::wait_staging(int set) {
    if (adm_pending[set]) {
        ECHK(this, hipEventSynchronize(ev_adm[set]));
        adm_pending[set] = false;
    }
    return OT_OK;
}

void BatchEngine::release(int k) {
    Slot& s = slots[k];
    if (!s.live) return;
    if (!s.finished) {
        --n_live_running;
        items_running -= s.parts_cap;
    }
    pool.release(s.mem);
    s = Slot{};
    free_slots.push_back(k);
    while (hi_slot > 0 && !slots[hi_slot - 1].live) --hi_slot;
}

ot_status BatchEngine::launch_chunk() {
    const int gi = gidx();
    if (ot_status st = capture(gi)) return st;
    ECHK(this, hipGraphLaunch(graph[gi], stream));
    ++chunks;
    return OT_OK;
}

// Takes a snapshot of the control blocks behind the work queued so far;
// with `wait`, also waits for the previous snapshot and marks every
// instance it shows done as finished (returned in `finished`).
ot_status BatchEngine::collect(bool wait, std::vector<int>& finished) {
    finished.clear();
    const int cur = snap_pending < 0 ? 0 : (snap_pending ^ 1);
    const int prev = snap_pending;
    const int hi = hi_slot;
    ECHK(this, hipMemcpyAsync(snap[cur], ctl, sizeof(Ctl) * std::max(hi, 1), hipMemcpyDeviceToHost, stream));
    ECHK(this, hipEventRecord(ev_snap[cur], stream));
    const int prev_hi = snap_hi;
    snap_pending = cur;
    snap_hi = hi;
    snap_seq[cur] = ++seq;
    if (!wait || prev < 0) return OT_OK;
    ECHK(this, hipEventSynchronize(ev_snap[prev]));
    apply_snapshot(prev, prev_hi, &finished);
    return OT_OK;
}

void BatchEngine::apply_snapshot(int which, int hi, std::vector<int>* finished) {
    for (int k = 0; k < hi; ++k) {
        Slot& s = slots[k];
        if (!s.live || s.finished || snap_seq[which] <= s.adm_seq) continue;
        const Ctl& c = snap[which][k];
        if (c.phase == kPhDone) {
            s.fin = c;
            s.finished = true;
            --n_live_running;
            items_running -= s.parts_cap;
            if (finished) finished->push_back(k);
        }
    }
}

// Waits for the newest snapshot and applies it.
ot_status BatchEngine::drain_snapshot(std::vector<int>* finished) {
    if (snap_pending < 0) return OT_OK;
    ECHK(this, hipEventSynchronize(ev_snap[snap_pending]));
    apply_snapshot(snap_pending, snap_hi, finished);
    return OT_OK;
}

// Rebuilds the parts of the given (not yet started) instances for another
// rows-per-part value and re-queues their first sweep items.
ot_status BatchEngine::relayout(const std::vector<int>& ks, int w, int64_t rpp) {
    for (int q = 0; q < 2; ++q)  // the relayout staging is reused only after admissions have landed
        if (ot_status st = wait_staging(q)) return st;
    waves = w;
    rpp_rows = rpp;
    int n_items = 0;
    const int n = (int)ks.size();
    for (int q = 0; q < n; ++q) {
        Slot& s = slots[ks[q]];
        s.d.rpp = rpp;
        s.d.parts = (int)parts_of(s.I, rpp);
        relay_h[q] = ks[q];
        relay_h[n + q] = n_items;
        n_items += s.d.parts;
    }
    ECHK(this, hipMemcpyAsync(relay_d, relay_h, sizeof(int) * 2 * n, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_bclear, dim3(1), dim3(64), 0, stream, L[0]);
    hipLaunchKernelGGL(k_brelayout, dim3(n), dim3(256), 0, stream, tab, (const int*)relay_d,
                       (const int*)(relay_d + n), rpp, L[0]);
    hipLaunchKernelGGL(k_bcount, dim3(1), dim3(64), 0, stream, L[0], n_items, n);
    ECHK(this, hipGetLastError());
    ECHK(this, hipStreamSynchronize(stream));
    return OT_OK;
}

// Autotuner cache, shared by every engine of the process: the chosen
// (waves, rows per part) per batch shape. A shape is the device (architecture
// and CU count) and the histogram of the instances' (ceil log2 I, ceil log2 J)
// buckets, with each bucket's count rounded up to a power of two, so that
// batches of similar sizes share an entry. When OT_ASSOC_TUNE_CACHE names a
// file, its entries ("shape waves rows_per_part" per line) are read before the
// first tuning with that path (they take precedence over choices made in this
// process) and every new choice is appended to it, so later processes make
// the same choice without timing anything.
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int64_t>> g_tune;
std::vector<std::string> g_tune_files;  // cache files read so far

bool tune_valid(int w, int64_t r) { return (w == 4 || w == 8) && (r == 64 || r == 128 || r == 256); }

void tune_load(const std::string& path) {
    if (std::find(g_tune_files.begin(), g_tune_files.end(), path) != g_tune_files.end()) return;
    g_tune_files.push_back(path);
    FILE* fp = std::fopen(path.c_str(), "r");
    if (!fp) return;
    char key[1024];
    int w = 0;
    long long r = 0;
    while (std::fscanf(fp, "%1023s %d %lld", key, &w, &r) == 3)
        if (key[0] != '#' && tune_valid(w, r)) g_tune[key] = {w, (int64_t)r};
    std::fclose(fp);
}

void tune_store(const std::string& path, const std::string& key, int w, int64_t r) {
    FILE* fp = std::fopen(path.c_str(), "a");
    if (!fp) return;  // (a cache that cannot be written is only a lost speed-up)
    std::fprintf(fp, "%s %d %lld\n", key.c_str(), w, (long long)r);
    std::fclose(fp);
}

int ceil_log2(int64_t x) {
    int k = 0;
    while (((int64_t)1 << k) < x) ++k;
    return k;
}
}  // namespace

std::string BatchEngine::tune_key(const std::vector<int>& ks) const {
    std::map<std::pair<int, int>, int> hist;
    for (int k : ks) ++hist[{ceil_log2(slots[k].I), ceil_log2(slots[k].J)}];
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, device);
    std::string key = std::string(prop.gcnArchName).substr(0, 16) + "/" + std::to_string(num_cu);
    for (const auto& e : hist) {
        key += "/" + std::to_string(e.first.first) + "." + std::to_string(e.first.second) + "x" +
               std::to_string(1 << ceil_log2(e.second));
    }
    for (char& c : key)
        if (c == ' ' || c == '\t' || c == '\n' || c == ':') c = '_';
    return key;
}

// Autotuner: times the first FP32 sweep of the admitted batch under each
// (workgroup waves, rows per part) candidate. The sweep reads f and g of
// parity 0 and writes only the other parity and partials, so the trial
// launches leave the starting state intact. The default (8, 128) is kept
// unless a candidate, tried in a fixed order, beats the best so far by 3 %
// in its median of five launches (timing noise then rarely flips a choice);
// a cached choice is taken without timing.
ot_status BatchEngine::tune(const std::vector<int>& ks) {
    const std::string key = tune_key(ks);
    const char* env = std::getenv("OT_ASSOC_TUNE_CACHE");
    const std::string path = env ? env : "";
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!path.empty()) tune_load(path);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            // admission already partitioned with the engine's current rows per part
            if (it->second.second == rpp_rows) {
                waves = it->second.first;
                return OT_OK;
            }
            return relayout(ks, it->second.first, it->second.second);
        }
    }
    hipEvent_t ev[6];
    for (auto& e : ev) ECHK(this, hipEventCreate(&e));
    float best = 0.0f;
    int bw = 8;
    int64_t br = 128;
    ot_status st = OT_OK;
    const std::pair<int, int64_t> cand[6] = {{8, 128}, {8, 64}, {8, 256}, {4, 64}, {4, 128}, {4, 256}};
    for (const auto& c : cand) {
        if ((st = relayout(ks, c.first, c.second))) break;
        const int wi = c.first == 4 ? 0 : 1;
        auto launch = [&]() {
            const BInst* T = tab;
            if (wi == 0)
                hipLaunchKernelGGL((k_bsweep<false, 4>), dim3(grid32[0]), dim3(256), lds32[0], stream, T,
                                   (const BItem*)L[0].it32, (const int*)L[0].cnt, L[1].cnt);
            else
                hipLaunchKernelGGL((k_bsweep<false, 8>), dim3(grid32[1]), dim3(512), lds32[1], stream, T,
                                   (const BItem*)L[0].it32, (const int*)L[0].cnt, L[1].cnt);
        };
        launch();  // warm-up
        hipEventRecord(ev[0], stream);
        for (int rep = 0; rep < 5; ++rep) {
            launch();
            hipEventRecord(ev[rep + 1], stream);
        }
        if (hipEventSynchronize(ev[5]) != hipSuccess) {
            st = fail(OT_EDEVICE, "tuning sweep failed");
            break;
        }
        float t[5];
        for (int rep = 0; rep < 5; ++rep) hipEventElapsedTime(&t[rep], ev[rep], ev[rep + 1]);
        std::sort(t, t + 5);
        const float med = t[2];
        if (best == 0.0f || med < 0.97f * best) {
            best = med;
            bw = c.first;
            br = c.second;
        }
    }
    for (auto& e : ev) hipEventDestroy(e);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto ins = g_tune.emplace(key, std::make_pair(bw, br));
        if (ins.second && !path.empty()) tune_store(path, key, bw, br);
        bw = ins.first->second.first;  // (another thread's choice for the same shape wins)
        br = ins.first->second.second;
    }
    return relayout(ks, bw, br);
}

static void fill_result(const Slot& s, ot_assoc_result* r) {
    const Ctl& c = s.fin;
    ot_status rs = OT_OK;
    if (c.numeric_bad == 2) rs = OT_EINVAL;  // marginals rejected on the device
    else if (c.numeric_bad || !std::isfinite(c.chk_violation)) rs = OT_ENUMERIC;
    else if (!(c.chk_violation < c.tol)) rs = OT_WARN_MAXITER;
    r->iterations = c.result_iter;
    r->fp64_iterations = c.fp64_iters;
    r->status = rs;
    r->flags = 0;
    r->marginal_violation = c.chk_violation;
    r->objective = c.chk_objective;
    r->reg_objective = c.chk_reg_objective;
    r->dual_objective = c.chk_dual;
    r->seconds = 0.0;
}

static ot_status slot_potentials(BatchEngine* e, const Slot& s, double* f, double* g, ot_mem mem) {
    const int par = s.fin.result_iter & 1;
    const hipMemcpyKind k = mem == OT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (f) ECHK(e, hipMemcpyAsync(f, s.d.f[par], sizeof(double) * s.I, k, e->stream));
    if (g) ECHK(e, hipMemcpyAsync(g, s.d.g[par], sizeof(double) * s.J, k, e->stream));
    ECHK(e, hipStreamSynchronize(e->stream));
    return OT_OK;
}

static ot_status slot_plan(BatchEngine* e, const Slot& s, void* pi, ot_mem mem, ot_dtype dtype) {
    const int par = s.fin.result_iter & 1;
    const size_t bytes = (size_t)s.I * s.J * (dtype == OT_F32 ? 4 : 8);
    void* dst = pi;
    char* tmp = nullptr;
    if (mem == OT_MEM_HOST) {
        tmp = e->pool.alloc(bytes);
        if (!tmp) return e->fail(OT_ENOMEM, "no device memory for the plan");
        dst = tmp;
    }
    const int nch = (s.J + 255) / 256;
    const size_t lds = sizeof(double) * (size_t)nch * 256;
    const int grid = (int)std::min<int64_t>(4096, (s.I + 7) / 8);
    const DenseSrc<float> src{s.d.C, s.d.ld};
    if (dtype == OT_F32)
        hipLaunchKernelGGL((k_plan<DenseSrc<float>, float, 4>), dim3(grid), dim3(512), lds, e->stream, (int64_t)0, s.I, s.J, nch,
                           (const double*)s.d.f[par], (const double*)s.d.g[par], (const SolveParams*)s.prm, (float*)dst, src);
    else
        hipLaunchKernelGGL((k_plan<DenseSrc<float>, double, 4>), dim3(grid), dim3(512), lds, e->stream, (int64_t)0, s.I, s.J, nch,
                           (const double*)s.d.f[par], (const double*)s.d.g[par], (const SolveParams*)s.prm, (double*)dst, src);
    ot_status st = OT_OK;
    hipError_t er = hipGetLastError();
    if (er != hipSuccess) st = e->fail(OT_EDEVICE, "plan launch failed: %s", hipGetErrorString(er));
    if (!st && tmp) {
        er = hipMemcpyAsync(pi, tmp, bytes, hipMemcpyDeviceToHost, e->stream);
        if (er != hipSuccess) st = e->fail(OT_EDEVICE, "plan copy failed: %s", hipGetErrorString(er));
    }
    er = hipStreamSynchronize(e->stream);
    if (!st && er != hipSuccess) st = e->fail(OT_EDEVICE, "plan failed: %s", hipGetErrorString(er));
    if (tmp) e->pool.release(tmp);
    return st;
}

static size_t default_budget(int device) {
    size_t fr = 0, tot = 0;
    if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)8 << 30;
    return std::min<size_t>((size_t)256 << 30, fr / 10 * 9);
}

// Runs chunks until every listed slot is finished. Chunk c + 1 is queued
// before the snapshot behind chunk c is read, so the device never idles on
// the host; max_chunks bounds the loop (every instance ends within
// max_iter + 2 iterations of its own, so this is only a guard).
static ot_status run_to_completion(BatchEngine* e, const std::vector<int>& ks, long max_chunks) {
    std::vector<int> fin;
    auto open_count = [&]() {
        int n = 0;
        for (int k : ks) n += e->slots[k].finished ? 0 : 1;
        return n;
    };
    for (long c = 0; c < max_chunks && open_count() > 0; ++c) {
        if (ot_status st = e->launch_chunk()) return st;
        if (ot_status st = e->collect(true, fin)) return st;
    }
    if (ot_status st = e->drain_snapshot(nullptr)) return st;
    if (open_count() > 0) return e->fail(OT_EDEVICE, "batch did not finish within %ld chunks", max_chunks);
    return OT_OK;
}

extern "C" {

ot_status ot_assoc_solve_batch(ot_assoc* h, int n, const ot_cost_desc* costs, const double* const* a,
                               const double* const* b, const double* eps, double tol, int32_t max_iter,
                               ot_assoc_result* out) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (n < 1 || !costs || !a || !b || !eps) {
        h->err = "n must be >= 1 and the arrays non-NULL";
        return OT_EINVAL;
    }
    if (hipSetDevice(h->device) != hipSuccess) {
        h->err = "hipSetDevice failed";
        return OT_EDEVICE;
    }
    if (!h->batch) {
        BatchEngine* e = new BatchEngine();
        ot_status st = e->init(h->device, h->stream, 4096, 1 << 20, default_budget(h->device));
        if (st) {
            h->err = e->err;
            delete e;
            return st;
        }
        h->batch = e;
    }
    BatchEngine* e = h->batch;
    e->err.clear();
    e->polish_iters = std::max(0, h->opt.polish_iters);
    // the previous batch's instances are released first
    if (e->n_live_running > 0) {
        h->err = "a batch is still running on this handle";
        return OT_ESTATE;
    }
    for (int k = 0; k < e->cap_slots; ++k)
        if (e->slots[k].live) e->release(k);
    if (n > e->cap_slots) {
        h->err = "batch larger than 4096 instances";
        return OT_EINVAL;
    }
    std::vector<AdmitReq> reqs((size_t)n);
    for (int q = 0; q < n; ++q) {
        reqs[q].cost = costs + q;
        reqs[q].a = a[q];
        reqs[q].b = b[q];
        reqs[q].eps = eps[q];
        reqs[q].tol = tol;
        reqs[q].max_iter = max_iter;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    std::vector<int> ks;
    ot_status st = e->admit(reqs, ks, true);
    if (!st) {
        // marginals were checked on the device: one read-back for all of them
        const int hi = *std::max_element(ks.begin(), ks.end()) + 1;
        if (hipMemcpyAsync(e->snap[0], e->ctl, sizeof(Ctl) * hi, hipMemcpyDeviceToHost, e->stream) != hipSuccess ||
            hipStreamSynchronize(e->stream) != hipSuccess)
            st = e->fail(OT_EDEVICE, "admission failed");
        for (size_t q = 0; q < ks.size() && !st; ++q)
            if (e->snap[0][ks[q]].numeric_bad == 2)
                st = e->fail(OT_EINVAL, "instance %zu: marginals must be positive, finite and balanced", q);
        if (st) {
            h->err = e->err;
            for (int k : ks) e->release(k);
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return st;
        }
    }
    if (!st && h->opt.batch_tune) st = e->tune(ks);
    if (!st && !h->opt.batch_tune) st = e->relayout(ks, 8, 128);
    if (!st) {
        hipEventRecord(e0, e->stream);
        st = run_to_completion(e, ks, (long)max_iter / kChunk + 16);
        hipEventRecord(e1, e->stream);
        hipEventSynchronize(e1);
    }
    float ms = 0.0f;
    if (!st) hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) {
        h->err = e->err;
        for (int k : ks) e->release(k);
        return st;
    }
    ot_status worst = OT_OK;
    for (int q = 0; q < n; ++q) {
        ot_assoc_result r{};
        fill_result(e->slots[ks[q]], &r);
        r.seconds = ms * 1e-3;
        if (out) out[q] = r;
        if (r.status < 0 && worst >= 0) worst = (ot_status)r.status;
        else if (r.status > 0 && worst == OT_OK) worst = (ot_status)r.status;
    }
    e->tab_order = ks;
    if (worst < 0) h->err = "an instance of the batch failed numerically";
    return worst;
}

ot_status ot_assoc_batch_config(ot_assoc* h, int* waves, int* rows_per_part) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    if (!h->batch) {
        h->err = "no batch has run on this handle";
        return OT_ESTATE;
    }
    if (waves) *waves = h->batch->waves;
    if (rows_per_part) *rows_per_part = (int)h->batch->rpp_rows;
    return OT_OK;
}

ot_status ot_assoc_batch_potentials(ot_assoc* h, int k, double* f, double* g, ot_mem mem) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    BatchEngine* e = h->batch;
    if (!e || k < 0 || k >= (int)e->tab_order.size()) {
        h->err = "no batched instance with that index";
        return e ? OT_EINVAL : OT_ESTATE;
    }
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) {
        h->err = "bad memory space";
        return OT_EINVAL;
    }
    const Slot& s = e->slots[e->tab_order[k]];
    if (!s.live || !s.finished) {
        h->err = "batched instance not available";
        return OT_ESTATE;
    }
    ot_status st = slot_potentials(e, s, f, g, mem);
    if (st) h->err = e->err;
    return st;
}

ot_status ot_assoc_batch_plan(ot_assoc* h, int k, void* pi, ot_mem mem, ot_dtype dtype) {
    if (!h) return OT_EINVAL;
    h->err.clear();
    BatchEngine* e = h->batch;
    if (!e || k < 0 || k >= (int)e->tab_order.size()) {
        h->err = "no batched instance with that index";
        return e ? OT_EINVAL : OT_ESTATE;
    }
    if (!pi || (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) || (dtype != OT_F32 && dtype != OT_F64)) {
        h->err = "bad plan buffer, memory space or dtype";
        return OT_EINVAL;
    }
    const Slot& s = e->slots[e->tab_order[k]];
    if (!s.live || !s.finished) {
        h->err = "batched instance not available";
        return OT_ESTATE;
    }
    ot_status st = slot_plan(e, s, pi, mem, dtype);
    if (st) h->err = e->err;
    return st;
}

}  // extern "C"

// ================================================================ serving ==
struct Resident {
    char* mem = nullptr;
    double* f = nullptr;
    double* g = nullptr;
    int64_t I = 0;
    int J = 0;
    long last_use = 0;
};

struct Pending {
    uint64_t ticket;
    ot_request req;
    double t_submit;
};

// Requests admitted together per admission call of the serving loop.
constexpr size_t kServeAdmitGroup = 64;

// Device-to-device copies of FP64 vectors passed by value: one launch for a
// whole set of resident-potential updates, one workgroup per copy.
constexpr int kCopyPairs = 32;
struct CopyPairs {
    const double* src[kCopyPairs];
    double* dst[kCopyPairs];
    int64_t cnt[kCopyPairs];
};
static __global__ __launch_bounds__(256) void k_copy_pairs(CopyPairs P) {
    const double* s = P.src[blockIdx.x];
    double* d = P.dst[blockIdx.x];
    for (int64_t e = threadIdx.x; e < P.cnt[blockIdx.x]; e += blockDim.x) d[e] = s[e];
}
struct PendingCopy {
    const double* src;
    double* dst;
    int64_t cnt;
};

struct ot_serve {
    BatchEngine eng;
    std::string err;
    uint64_t next_ticket = 1;
    long tick = 0;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Resident> resident;
    std::deque<ot_completion> done;
    int keep_layouts = 4096;
    std::vector<int> running;  // slots in flight
    std::unordered_map<int, int> warm_of;  // slot -> 1 if warm started
    std::unordered_map<int, uint64_t> pinned_key;
    std::vector<PendingCopy> copies;  // resident updates not yet queued
};

// Queues the pending resident updates on the engine stream.
static ot_status flush_copies(ot_serve* s) {
    BatchEngine& e = s->eng;
    for (size_t q0 = 0; q0 < s->copies.size(); q0 += kCopyPairs) {
        CopyPairs P{};
        const int n = (int)std::min<size_t>(kCopyPairs, s->copies.size() - q0);
        for (int q = 0; q < n; ++q) {
            P.src[q] = s->copies[q0 + q].src;
            P.dst[q] = s->copies[q0 + q].dst;
            P.cnt[q] = s->copies[q0 + q].cnt;
        }
        hipLaunchKernelGGL(k_copy_pairs, dim3(n), dim3(256), 0, e.stream, P);
    }
    s->copies.clear();
    ECHK(&e, hipGetLastError());
    return OT_OK;
}

static ot_status serve_fail(ot_serve* s, ot_status st, const std::string& m) {
    s->err = m;
    return st;
}

// Copies a finished slot's potentials into the resident set of its layout.
static ot_status keep_resident(ot_serve* s, const Slot& sl) {
    BatchEngine& e = s->eng;
    Resident& r = s->resident[sl.layout_key];
    // (an admission copies from a resident set on the same stream before any
    // later update or reuse of its memory, so no set is ever pinned)
    if (r.mem && (r.I != sl.I || r.J != sl.J)) {
        if (ot_status st = flush_copies(s)) return st;  // nothing pending may target freed memory
        e.pool.release(r.mem);
        r = Resident{};
    }
    if (!r.mem) {
        r.mem = e.pool.alloc(align_up(sizeof(double) * sl.I) + align_up(sizeof(double) * sl.J));
        if (!r.mem) {
            s->resident.erase(sl.layout_key);
            return OT_OK;  // no room: the layout will start cold next time
        }
        r.f = (double*)r.mem;
        r.g = (double*)(r.mem + align_up(sizeof(double) * sl.I));
        r.I = sl.I;
        r.J = sl.J;
    }
    const int par = sl.fin.result_iter & 1;
    // the latest completion of a layout wins (pending copies run together)
    s->copies.erase(std::remove_if(s->copies.begin(), s->copies.end(),
                                   [&](const PendingCopy& c) { return c.dst == r.f || c.dst == r.g; }),
                    s->copies.end());
    s->copies.push_back(PendingCopy{sl.d.f[par], r.f, sl.I});
    s->copies.push_back(PendingCopy{sl.d.g[par], r.g, sl.J});
    r.last_use = ++s->tick;
    return OT_OK;
}

// Frees the least recently used resident set that no admission still reads.
static bool evict_one(ot_serve* s, uint64_t keep_key) {
    auto victim = s->resident.end();
    for (auto it = s->resident.begin(); it != s->resident.end(); ++it) {
        if (it->first == keep_key) continue;
        if (victim == s->resident.end() || it->second.last_use < victim->second.last_use) victim = it;
    }
    if (victim == s->resident.end()) return false;
    if (flush_copies(s)) return false;  // nothing pending may target freed memory
    s->eng.pool.release(victim->second.mem);
    s->resident.erase(victim);
    return true;
}

extern "C" {

double ot_serve_now(void) { return now_s(); }

ot_status ot_serve_default_options(ot_serve_options* o) {
    if (!o) return OT_EINVAL;
    std::memset(o, 0, sizeof *o);
    o->polish_iters = 1;
    o->sweep_waves = 8;
    o->rows_per_part = 128;
    return OT_OK;
}

ot_status ot_serve_create(ot_serve** out, const ot_serve_options* opt) {
    if (!out) return OT_EINVAL;
    *out = nullptr;
    ot_serve_options o;
    ot_serve_default_options(&o);
    if (opt) o = *opt;
    if (o.max_slots < 0 || o.max_items < 0 || o.polish_iters < 0 || o.budget_bytes < 0) return OT_EINVAL;
    if (o.sweep_waves != 0 && o.sweep_waves != 4 && o.sweep_waves != 8) return OT_EINVAL;
    if (o.rows_per_part != 0 && o.rows_per_part != 64 && o.rows_per_part != 128 && o.rows_per_part != 256)
        return OT_EINVAL;
    ot_serve* s = new ot_serve();
    const size_t budget = o.budget_bytes > 0 ? (size_t)o.budget_bytes : default_budget(o.device);
    ot_status st = s->eng.init(o.device, (hipStream_t)o.stream, o.max_slots ? o.max_slots : 1024,
                               o.max_items ? o.max_items : (1 << 19), budget);
    if (st) {
        delete s;
        return st;
    }
    s->eng.polish_iters = o.polish_iters;
    s->eng.waves = o.sweep_waves ? o.sweep_waves : 8;
    s->eng.rpp_rows = o.rows_per_part ? o.rows_per_part : 128;
    s->keep_layouts = o.keep_layouts > 0 ? o.keep_layouts : 4096;
    *out = s;
    return OT_OK;
}

const char* ot_serve_last_error(const ot_serve* s) { return s ? s->err.c_str() : ""; }

ot_status ot_serve_submit(ot_serve* s, const ot_request* r, uint64_t* ticket) {
    if (!s) return OT_EINVAL;
    s->err.clear();
    if (!r || !r->a || !r->b) return serve_fail(s, OT_EINVAL, "request or marginals are NULL");
    if (ot_status st = check_desc(&s->eng, &r->cost)) return serve_fail(s, st, s->eng.err);
    if (!(r->eps > 0.0) || !std::isfinite(r->eps) || !(r->tol >= 0.0) || r->max_iter < 1)
        return serve_fail(s, OT_EINVAL, "bad eps, tol or max_iter");
    Pending p{s->next_ticket++, *r, now_s()};
    s->queue.push_back(p);
    if (ticket) *ticket = p.ticket;
    return OT_OK;
}

// Admits from the head of the queue while slots, work-list room and the
// byte budget allow (evicting idle resident potentials if that makes room),
// runs one chunk when anything is in flight, and hands back completions.
ot_status ot_serve_progress(ot_serve* s, ot_completion* out, int max_out, int* n_out) {
    if (!s) return OT_EINVAL;
    s->err.clear();
    if (n_out) *n_out = 0;
    BatchEngine& e = s->eng;
    if (hipSetDevice(e.device) != hipSuccess) return serve_fail(s, OT_EDEVICE, "hipSetDevice failed");
    // 1. admission, in groups from the head of the queue: one staging copy
    // and one set of admission launches per group. A group whose admission
    // fails is retried one request at a time, so that the error completes
    // the request it belongs to.
    size_t gmax = kServeAdmitGroup;
    auto complete_with = [&](const Pending& p, ot_status st) {
        ot_completion c{};
        c.ticket = p.ticket;
        c.user_tag = p.req.user_tag;
        c.layout_key = p.req.layout_key;
        c.t_submit = p.t_submit;
        c.t_admit = c.t_done = now_s();
        c.result.status = st;
        s->done.push_back(c);
    };
    while (!s->queue.empty()) {
        std::vector<AdmitReq> group;
        std::vector<Resident*> gres;
        for (size_t q = 0; q < s->queue.size() && group.size() < gmax; ++q) {
            const Pending& p = s->queue[q];
            AdmitReq ar;
            ar.cost = &p.req.cost;
            ar.a = p.req.a;
            ar.b = p.req.b;
            ar.eps = p.req.eps;
            ar.tol = p.req.tol;
            ar.max_iter = p.req.max_iter;
            Resident* res = nullptr;
            if (p.req.layout_key) {
                auto it = s->resident.find(p.req.layout_key);
                if (it != s->resident.end() && it->second.I == p.req.cost.I && it->second.J == p.req.cost.J) {
                    res = &it->second;
                    ar.f0 = res->f;
                    ar.g0 = res->g;
                }
            }
            group.push_back(ar);
            gres.push_back(res);
        }
        std::vector<int> ks;
        ot_status st = e.admit(group, ks, false);
        if (st) {
            if (group.size() > 1) {
                gmax = 1;
                continue;
            }
            // a request the engine rejects is completed with its error
            complete_with(s->queue.front(), st);
            s->queue.pop_front();
            gmax = kServeAdmitGroup;
            continue;
        }
        gmax = kServeAdmitGroup;
        if (ks.empty()) {
            if (evict_one(s, s->queue.front().req.layout_key)) continue;  // retry with more room
            if (e.n_live_running > 0) break;                               // wait for running requests to finish
            complete_with(s->queue.front(), OT_ENOMEM);  // it cannot fit even on an idle engine
            s->queue.pop_front();
            continue;
        }
        for (size_t q = 0; q < ks.size(); ++q) {
            const Pending& p = s->queue.front();
            Slot& sl = e.slots[ks[q]];
            sl.ticket = p.ticket;
            sl.user_tag = p.req.user_tag;
            sl.layout_key = p.req.layout_key;
            sl.t_submit = p.t_submit;
            s->warm_of[ks[q]] = gres[q] ? 1 : 0;
            if (gres[q]) gres[q]->last_use = ++s->tick;
            s->running.push_back(ks[q]);
            s->queue.pop_front();
        }
    }
    // 2. one chunk, and the snapshot behind the previous one
    std::vector<int> fin;
    if (e.n_live_running > 0) {
        if (ot_status st = e.launch_chunk()) return serve_fail(s, st, e.err);
        if (ot_status st = e.collect(true, fin)) return serve_fail(s, st, e.err);
    } else if (e.snap_pending >= 0) {
        if (ot_status st = e.drain_snapshot(&fin)) return serve_fail(s, st, e.err);
        e.snap_pending = -1;
    }
    // 3. completions: keep the layouts' potentials, then free the slots (once
    // the resident copies that read them are queued, so that no slot memory
    // is handed out again while a pending copy still reads it)
    const double t = now_s();
    for (int k : fin) {
        Slot& sl = e.slots[k];
        ot_completion c{};
        c.ticket = sl.ticket;
        c.user_tag = sl.user_tag;
        c.layout_key = sl.layout_key;
        c.warm = s->warm_of[k];
        c.t_submit = sl.t_submit;
        c.t_admit = sl.t_admit;
        c.t_done = t;
        fill_result(sl, &c.result);
        if (sl.layout_key && c.result.status >= 0) {
            if ((int)s->resident.size() >= s->keep_layouts && !s->resident.count(sl.layout_key)) evict_one(s, 0);
            if (ot_status st = keep_resident(s, sl)) return serve_fail(s, st, e.err);
        }
        s->warm_of.erase(k);
        s->running.erase(std::remove(s->running.begin(), s->running.end(), k), s->running.end());
        s->done.push_back(c);
    }
    if (ot_status st = flush_copies(s)) return serve_fail(s, st, e.err);
    for (int k : fin) e.release(k);
    int n = 0;
    while (n < max_out && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    if (n_out) *n_out = n;
    return OT_OK;
}

ot_status ot_serve_counts(const ot_serve* s, int* queued, int* running, int* resident, double* bytes_in_use) {
    if (!s) return OT_EINVAL;
    if (queued) *queued = (int)s->queue.size();
    if (running) *running = (int)s->running.size();
    if (resident) *resident = (int)s->resident.size();
    if (bytes_in_use) *bytes_in_use = (double)s->eng.pool.in_use;
    return OT_OK;
}

ot_status ot_serve_potentials(ot_serve* s, uint64_t layout_key, double* f, double* g, ot_mem mem) {
    if (!s) return OT_EINVAL;
    s->err.clear();
    auto it = s->resident.find(layout_key);
    if (it == s->resident.end()) return serve_fail(s, OT_ESTATE, "no resident potentials for that layout");
    if (mem != OT_MEM_HOST && mem != OT_MEM_DEVICE) return serve_fail(s, OT_EINVAL, "bad memory space");
    BatchEngine& e = s->eng;
    const hipMemcpyKind k = mem == OT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (f && hipMemcpyAsync(f, it->second.f, sizeof(double) * it->second.I, k, e.stream) != hipSuccess)
        return serve_fail(s, OT_EDEVICE, "copy failed");
    if (g && hipMemcpyAsync(g, it->second.g, sizeof(double) * it->second.J, k, e.stream) != hipSuccess)
        return serve_fail(s, OT_EDEVICE, "copy failed");
    if (hipStreamSynchronize(e.stream) != hipSuccess) return serve_fail(s, OT_EDEVICE, "copy failed");
    return OT_OK;
}

void ot_serve_destroy(ot_serve* s) { delete s; }

}  // extern "C"
