// The solver handle shared by the single-instance and the batched entry
// points of the library (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/ot_assoc.h"
#include "cost_sources.h"
#include "device_common.h"

namespace otk_host {
struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};

// Device allocations of the library go through these, which count them
// (ot_assoc_device_allocations reports the count).
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_free(void* p);
}  // namespace otk_host

// Constants of the geometry cost functor (relative gains, log2-domain
// shadowing, median-normalised cost scale) from the public descriptor.
inline otk::GeoConst geo_const(const ot_geometry& g, double scale) {
    otk::GeoConst k{};
    k.alpha_half = 0.5 * g.pathloss_exp;
    k.shadow_c = g.shadow_sigma_db * std::log2(10.0) / 10.0;
    k.dmin2 = g.min_dist_m * g.min_dist_m;
    k.cscale = std::log(2.0) / (g.bandwidth_hz * scale);
    k.n0n = g.noise_w / (g.tx_power_w * g.ref_gain);
    k.key = g.shadow_key;
    return k;
}

struct BatchEngine;
void batch_engine_destroy(BatchEngine* e);
struct SnapState;
void snap_state_destroy(SnapState* s);

struct ot_assoc {
    int device = 0;
    int num_cu = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ot_assoc_options opt{};
    int64_t I_max = 0, J_max = 0;
    // device workspace
    double *a = nullptr, *b = nullptr;
    double* la = nullptr;  // ln a_i of the current instance (written by the solve's set-up)
    double *f[2] = {nullptr, nullptr}, *g[2] = {nullptr, nullptr};
    double *col_part = nullptr, *res_part = nullptr, *stat_part = nullptr;
    double* cpart = nullptr;  // per-column-group partials of the check
    otk::Ctl* ctl = nullptr;
    otk::SolveParams* prm = nullptr;
    int* bad = nullptr;
    unsigned long long* hist = nullptr;
    double* xch = nullptr;     // exchange block of the cooperative FP32 phase
    double* loads = nullptr;   // J_max: RRH loads summed by the last check (when fused)
    int lds_max = 0;           // LDS bytes a workgroup may allocate
    bool xch_zeroed = false;       // this solve's init launch zeroed the exchange block
    bool stop_recorded = false;    // ev_stop was recorded with the last control-block copy
    bool last_persistent = false;  // the last solve's FP32 phase was one cooperative launch
    int last_fast_iters = 0;       // ... and the FP32 iterations it ran
    hipEvent_t ev_coop[2] = {nullptr, nullptr};  // around that launch
    float* xy_dev = nullptr;  // I_max x 2
    float* xy_rrh = nullptr;  // J_max x 2
    double *s_all = nullptr, *s_ex = nullptr;
    int* j1 = nullptr;
    void* stage = nullptr;  // host-memory dense / rate matrices are copied here
    size_t stage_bytes = 0;
    bool stage_in_ws = false;  // the stage is the tail of a caller's workspace (never freed or grown)
    void* ws = nullptr;        // the single device block all fixed buffers are carved from
    void* work = nullptr;      // 2 (I_max + J_max) doubles of per-call work space (plan blocks, timers, Alg. 2)
    bool ws_owned = false;     // allocated by the library (else the caller's workspace)
    // pinned host mirrors
    otk::Ctl* ctl_h = nullptr;  // 2 slots
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_slot[2] = {nullptr, nullptr};
    std::vector<otk_host::GraphEntry> graphs;
    // state of the last solve
    bool solved = false;
    bool have_pot = false;
    int64_t I = 0, J = 0;
    int res_par = 0;  // parity of the buffers holding the returned iterate
    bool want_loads = false;   // checks also sum the RRH loads into `loads` (Alg. 2's solves)
    bool loads_fresh = false;  // the last check did, for the potentials it checked
    bool loads_valid = false;  // `loads` holds the loads of the returned potentials
    void* plan_out = nullptr;  // device plan the checks write (ot_assoc_set_plan_output), or null
    int plan_dtype = 0;        // OT_F32 / OT_F64 of plan_out
    int64_t plan_cap = 0;      // its elements
    bool plan_fresh = false;   // the last check wrote plan_out for the potentials it checked
    bool plan_valid = false;   // plan_out holds the plan of the returned potentials
    double eps = 0.0;
    ot_cost_desc last{};       // descriptor of the retained cost (pointers below replace the caller's)
    const void* cost_dev = nullptr;  // device copy (host inputs) or the caller's device matrix
    bool retained = false;     // the handle still holds the cost of the last solve
    std::string err;
    char* err_fixed = nullptr;  // if set, errors are written here (512 bytes) instead of `err`
    BatchEngine* batch = nullptr;  // engine of ot_assoc_solve_batch, created on first use
    SnapState* snap = nullptr;     // buffers and results of the last snapshot solve
};
