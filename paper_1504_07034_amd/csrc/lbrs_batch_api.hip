// C ABI of the ragged 1D batch (declared in include/lbrs.h): the plan (unit
// offsets, team sizes, list schedule of member jobs over the persistent
// grid), the scratch layout, and the graph-captured launch.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "lbrs.h"
#include "lbrs_launch.hpp"

using namespace lbrs;

struct lbrs_batch {
    int nunits, Q;
    long long total;
    int chunk, threads, grid;
    std::vector<long long> off;
    Unit1D* d_units;
    UnitState1D* d_states;
    unsigned* d_counters;
    long long* d_slot_off;
    EdgeSlot* d_slots;
    Job1D* d_jobs;
    int* d_job_begin;
    double* d_f;
    hipStream_t stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_steps;
};

namespace {

struct Plan {
    std::vector<long long> off;
    std::vector<Unit1D> units;
    std::vector<long long> slot_off;
    long long nslots = 0;
    std::vector<Job1D> jobs;
    std::vector<int> job_begin;
    size_t bytes[7];
    size_t total_bytes = 0;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int check_unit(const lbrs_params* p, int model) {
    if (p->model != model || p->law != LBRS_LAW_EULER || p->solid) return LBRS_E_INVAL;
    if (p->model == LBRS_D2Q4 || p->nx < 3 || p->ny != 1) return LBRS_E_INVAL;
    if (!(p->x1 > p->x0) || !(p->gamma > 1.0) || !(p->omega > 0.0 && p->omega < 2.0)) return LBRS_E_INVAL;
    if (p->bc[0] == LBRS_BC_WALL || p->bc[1] == LBRS_BC_WALL) return LBRS_E_INVAL;
    if ((p->bc[0] == LBRS_BC_PERIODIC) != (p->bc[1] == LBRS_BC_PERIODIC)) return LBRS_E_INVAL;
    if (p->bc[0] < 0 || p->bc[0] > 2 || p->bc[1] < 0 || p->bc[1] > 2) return LBRS_E_INVAL;
    if (p->lambda_mode < LBRS_LAMBDA_PER_STEP || p->lambda_mode > LBRS_LAMBDA_USER) return LBRS_E_INVAL;
    if (p->lambda_mode == LBRS_LAMBDA_USER && !(p->lambda_user > 0.0)) return LBRS_E_INVAL;
    if (p->lambda_mode != LBRS_LAMBDA_USER && !(p->cfl > 0.0 && p->cfl <= cfl_limit(p->model)))
        return LBRS_E_INVAL;
    return LBRS_OK;
}

void schedule_jobs(const std::vector<double>& work, int grid, Plan& P);

int make_plan(int nunits, const lbrs_params* units, const double* t_end, int chunk, int grid, Plan& P) {
    if (nunits < 1 || !units || chunk < 3 || grid < 1) return LBRS_E_INVAL;
    const int model = units[0].model;
    P.off.assign(nunits + 1, 0);
    P.units.resize(nunits);
    P.slot_off.resize(nunits);
    std::vector<double> work(nunits);
    int gmax = 0;
    for (int b = 0; b < nunits; ++b) {
        int rc = check_unit(&units[b], model);
        if (rc) return rc;
        double te = t_end ? t_end[b] : INFINITY;
        if (isnan(te)) return LBRS_E_INVAL;
        Unit1D& u = P.units[b];
        u.off = P.off[b];
        u.n = units[b].nx;
        u.periodic = units[b].bc[0] == LBRS_BC_PERIODIC;
        u.g = (u.n + chunk - 1) / chunk;
        u.lam_mode = units[b].lambda_mode == LBRS_LAMBDA_PER_STEP ? LAM_PER_STEP
                     : (units[b].lambda_mode == LBRS_LAMBDA_USER ? LAM_USER : LAM_FROZEN);
        u.dx = (units[b].x1 - units[b].x0) / u.n;
        u.gamma = units[b].gamma;
        u.omega = units[b].omega;
        u.cfl = units[b].cfl;
        u.t_end = te;
        u.lam_fixed = units[b].lambda_user;
        P.off[b + 1] = P.off[b] + u.n;
        P.slot_off[b] = P.nslots;
        P.nslots += 2LL * u.g;
        gmax = std::max(gmax, u.g);
        // relative work of a member before the lattice speeds are known:
        // steps ~ t_end * n / (cfl * L), times its cells
        double steps = isfinite(te) ? te * u.n / ((units[b].cfl > 0 ? units[b].cfl : 1.0) *
                                                  (units[b].x1 - units[b].x0))
                                    : 1.0;
        work[b] = steps * (double)((u.n + u.g - 1) / u.g) + 1.0;
    }
    if (gmax > grid || gmax > MAXTEAM) return LBRS_E_INVAL;  // a team must be co-resident
    schedule_jobs(work, grid, P);
    P.bytes[0] = align256(sizeof(Unit1D) * nunits);
    P.bytes[1] = align256(sizeof(UnitState1D) * nunits);
    P.bytes[2] = align256(sizeof(unsigned) * COUNTER_STRIDE * (size_t)nunits);
    P.bytes[3] = align256(sizeof(long long) * nunits);
    P.bytes[4] = align256(sizeof(EdgeSlot) * (size_t)P.nslots);
    P.bytes[5] = align256(sizeof(Job1D) * P.jobs.size());
    P.bytes[6] = align256(sizeof(int) * (grid + 1));
    P.total_bytes = 0;
    for (int i = 0; i < 7; ++i) P.total_bytes += P.bytes[i];
    return LBRS_OK;
}

// List schedule of the member jobs over the persistent workgroups: largest
// work first, each team on the earliest-free workgroups (starting together).
void schedule_jobs(const std::vector<double>& work, int grid, Plan& P) {
    const int nunits = (int)P.units.size();
    std::vector<int> order(nunits);
    for (int b = 0; b < nunits; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    std::vector<double> free_at(grid, 0.0);
    std::vector<std::vector<Job1D>> per(grid);
    std::vector<int> idx(grid);
    for (int b : order) {
        const Unit1D& u = P.units[b];
        for (int w = 0; w < grid; ++w) idx[w] = w;
        std::partial_sort(idx.begin(), idx.begin() + u.g, idx.end(), [&](int x, int y) {
            return free_at[x] < free_at[y] || (free_at[x] == free_at[y] && x < y);
        });
        double start = 0.0;
        for (int m = 0; m < u.g; ++m) start = std::max(start, free_at[idx[m]]);
        for (int m = 0; m < u.g; ++m) {
            Job1D j;
            j.unit = b;
            j.member = m;
            j.c0 = (int)((long long)m * u.n / u.g);
            j.c1 = (int)((long long)(m + 1) * u.n / u.g);
            per[idx[m]].push_back(j);
            free_at[idx[m]] = start + work[b];
        }
    }
    P.job_begin.assign(grid + 1, 0);
    P.jobs.clear();
    for (int w = 0; w < grid; ++w) {
        P.job_begin[w + 1] = P.job_begin[w] + (int)per[w].size();
        P.jobs.insert(P.jobs.end(), per[w].begin(), per[w].end());
    }
}

int default_threads(int chunk) {
    // chunk + 2 local cells over at most 4 cells per thread
    int w = chunk + 2;
    for (int t : {256, 512, 768, 1024})
        if (w <= t * 4 && (w + t - 1) / t <= 4 && t >= (w + 3) / 4) return t;
    return 1024;
}

int grid_for(int Q, int chunk, int threads) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (batch1d_lds_bytes(chunk) > prop.sharedMemPerBlock) return 0;
    int bpc = batch1d_blocks_per_cu(Q, threads, chunk);
    return bpc * prop.multiProcessorCount;
}

}  // namespace

extern "C" {

int lbrs_batch_query(int nunits, const lbrs_params* units, int chunk, long long* offsets,
                     size_t* scratch_bytes) {
    if (nunits < 1 || !units) return LBRS_E_INVAL;
    for (int b = 0; b < nunits; ++b)  // before the occupancy query asks the GPU
        if (check_unit(&units[b], units[0].model)) return LBRS_E_INVAL;
    const int Q = units[0].model == LBRS_D1Q2 ? 2 : 3;
    const int threads = default_threads(chunk);
    const int grid = grid_for(Q, chunk, threads);
    if (grid < 1) return LBRS_E_INVAL;
    Plan P;
    int rc = make_plan(nunits, units, nullptr, chunk, grid, P);
    if (rc) return rc;
    if (offsets)
        for (int b = 0; b <= nunits; ++b) offsets[b] = P.off[b];
    if (scratch_bytes) *scratch_bytes = P.total_bytes;
    return LBRS_OK;
}

int lbrs_batch_init(lbrs_batch** out, int nunits, const lbrs_params* units, const double* t_end,
                    int chunk, const double* d_U0, double* d_f, void* d_scratch, void* hip_stream) {
    if (!out) return LBRS_E_INVAL;
    *out = nullptr;
    if (nunits < 1 || !units || !d_U0 || !d_f || !d_scratch) return LBRS_E_INVAL;
    if (((uintptr_t)d_scratch & 255u) != 0) return LBRS_E_INVAL;
    const int Q = units[0].model == LBRS_D1Q2 ? 2 : 3;
    const int threads = default_threads(chunk);
    const int grid = grid_for(Q, chunk, threads);
    if (grid < 1) return LBRS_E_INVAL;
    Plan P;
    int rc = make_plan(nunits, units, t_end, chunk, grid, P);
    if (rc) return rc;
    lbrs_batch* b = new (std::nothrow) lbrs_batch();
    if (!b) return LBRS_E_NOMEM;
    b->nunits = nunits;
    b->Q = Q;
    b->total = P.off[nunits];
    b->chunk = chunk;
    b->threads = threads;
    b->grid = grid;
    b->off = P.off;
    char* s = (char*)d_scratch;
    b->d_units = (Unit1D*)s;
    s += P.bytes[0];
    b->d_states = (UnitState1D*)s;
    s += P.bytes[1];
    b->d_counters = (unsigned*)s;
    s += P.bytes[2];
    b->d_slot_off = (long long*)s;
    s += P.bytes[3];
    b->d_slots = (EdgeSlot*)s;
    s += P.bytes[4];
    b->d_jobs = (Job1D*)s;
    s += P.bytes[5];
    b->d_job_begin = (int*)s;
    b->d_f = d_f;
    b->stream = (hipStream_t)hip_stream;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_steps = -1;
    hipStream_t st = b->stream;
    bool ok = hipMemcpyAsync(b->d_units, P.units.data(), sizeof(Unit1D) * nunits, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(b->d_slot_off, P.slot_off.data(), sizeof(long long) * nunits, hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) ok = launch_batch1d_init(b->d_units, b->d_units, nunits, d_U0, d_f, b->total, b->d_states, Q, st) == hipSuccess;
    // Reschedule with the initial lattice speeds: a unit takes about
    // t_end * lambda_0 * n / L steps (lambda_0 = lambda*(U0)/cfl or the
    // user's speed), each member's work is that times its cells.
    std::vector<UnitState1D> s0(nunits);
    if (ok) ok = hipMemcpyAsync(s0.data(), b->d_states, sizeof(UnitState1D) * nunits, hipMemcpyDeviceToHost, st) == hipSuccess &&
                 hipStreamSynchronize(st) == hipSuccess;
    if (ok) {
        std::vector<double> work(nunits);
        for (int u = 0; u < nunits; ++u) {
            const Unit1D& un = P.units[u];
            const double L = un.dx * un.n;
            const double lam = isfinite(s0[u].lam_used) && s0[u].lam_used > 0.0 ? s0[u].lam_used : 1.0;
            const double steps = isfinite(un.t_end) ? un.t_end * lam * un.n / L : 1.0;
            work[u] = steps * (double)((un.n + un.g - 1) / un.g) + 1.0;
        }
        schedule_jobs(work, grid, P);
        ok = hipMemcpyAsync(b->d_jobs, P.jobs.data(), sizeof(Job1D) * P.jobs.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
             hipMemcpyAsync(b->d_job_begin, P.job_begin.data(), sizeof(int) * (grid + 1), hipMemcpyHostToDevice, st) == hipSuccess;
    }
    // the host plan must outlive the asynchronous copies
    if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        delete b;
        return LBRS_E_HIP;
    }
    *out = b;
    return LBRS_OK;
}

static hipError_t enqueue_run(lbrs_batch* b, int max_steps) {
    Batch1DArgs a;
    a.units = b->d_units;
    a.states = b->d_states;
    a.jobs = b->d_jobs;
    a.job_begin = b->d_job_begin;
    a.counters = b->d_counters;
    a.slots = b->d_slots;
    a.slot_off = b->d_slot_off;
    a.f = b->d_f;
    a.total = b->total;
    a.Q = b->Q;
    a.max_steps = max_steps;
    a.spin_limit = 1u << 27;
    hipError_t e = launch_zero_counters(b->d_counters, b->nunits, b->stream);
    if (e != hipSuccess) return e;
    return launch_batch1d(a, b->grid, b->threads, b->chunk, b->stream);
}

int lbrs_batch_run(lbrs_batch* b, int max_steps) {
    if (!b || max_steps < 0) return LBRS_E_INVAL;
    if (max_steps == 0) return LBRS_OK;
    // the counter reset and the persistent launch, captured once per step cap
    if (b->graph_steps != max_steps) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->graph_steps = -1;
        hipStream_t cap;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return LBRS_E_HIP;
        hipStream_t keep = b->stream;
        b->stream = cap;
        bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) ok = enqueue_run(b, max_steps) == hipSuccess;
        hipGraph_t g = nullptr;
        ok = (hipStreamEndCapture(cap, &g) == hipSuccess) && ok;
        b->stream = keep;
        (void)hipStreamDestroy(cap);
        if (!ok || hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return LBRS_E_HIP;
        }
        b->graph = g;
        b->graph_steps = max_steps;
    }
    return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? LBRS_OK : LBRS_E_HIP;
}

int lbrs_batch_get_state(lbrs_batch* b, double* t, long long* nsteps, double* lambda,
                         unsigned* status, long long* fail_step) {
    if (!b) return LBRS_E_INVAL;
    std::vector<UnitState1D> h(b->nunits);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LBRS_E_HIP;
    if (hipMemcpy(h.data(), b->d_states, sizeof(UnitState1D) * b->nunits, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return LBRS_E_HIP;
    int rc = LBRS_OK;
    for (int u = 0; u < b->nunits; ++u) {
        if (t) t[u] = h[u].t;
        if (nsteps) nsteps[u] = h[u].nsteps;
        if (lambda) lambda[u] = h[u].lam_used;
        if (status) status[u] = h[u].status;
        if (fail_step) fail_step[u] = h[u].fail_step;
        if (h[u].status & 2u) rc = LBRS_E_HIP;
        else if ((h[u].status & 1u) && rc == LBRS_OK) rc = LBRS_E_NONPHYSICAL;
    }
    return rc;
}

int lbrs_batch_moments(lbrs_batch* b, double* d_U) {
    if (!b || !d_U) return LBRS_E_INVAL;
    CellArgs a;
    a.plane = b->total;
    a.ps = b->total;
    a.rs = b->total;
    a.nx = (int)std::min<long long>(b->total, 0x7fffffff);
    a.ny = 1;
    a.model = b->Q == 2 ? LBRS_D1Q2 : LBRS_D1Q3;
    a.gamma = 1.4;
    // a 1D pool with plane stride `total` is one row of `total` cells
    if (b->total > 0x7fffffff) return LBRS_E_INVAL;
    return launch_pool_moments(a, b->d_f, d_U, b->stream) == hipSuccess ? LBRS_OK : LBRS_E_HIP;
}

void lbrs_batch_destroy(lbrs_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"
