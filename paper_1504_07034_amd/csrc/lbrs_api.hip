// C ABI of the LBRS library (declared in include/lbrs.h): parameter checks,
// the context, and the launch sequence of every call.  No call allocates
// device memory; all large buffers are the caller's.
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include "lbrs.h"
#include "lbrs_launch.hpp"


using namespace lbrs;

struct lbrs_ctx {
    lbrs_params P;
    int Q, K, dim;
    long long plane;
    long long ps, rs;    // population offset p*ps + y*rs + x
    double dx;
    double* f0;
    double* f1;
    DevState* st;
    hipStream_t stream;
    long long launches;  // step launches since the last (re)initialisation
    int rows_per_tile;   // 0: automatic (one balanced round of resident waves)
    int waves_per_block;
    int alternate;       // 2D: odd row segments march upwards (mirrored view)
    int persistent_max;  // largest 1D domain run by the persistent kernel
    int cu_count;
    int bpc[2][2][17];   // resident step-kernel workgroups per CU, by (alternate, dirichlet, waves)
    bool dir;            // some side is DIRICHLET
    int sbpc[17];        // resident scalar-step workgroups per CU, by waves per block
    unsigned short* codes;  // body node codes in the scratch area (null: no body)
    int fuse;            // 2D Euler: time steps per launch (1, or 2 to 4 fused)
    bool rounds;         // fused PER_STEP calls may wait between rounds of launches
    long long pair_enq;  // fused step launches enqueued since init (idle ones included)
    void* hst;           // pinned host copy of the time state and the call's step limit
                         // (fused PER_STEP rounds), or null
    PairState* pst;      // record of the fused launches (scratch area, behind the time state)
    PredCand* cand;      // candidate list of the per-step prediction (scratch area), or null
    int pbpc[3][KMAX_STEPS + 1][17];  // resident fused-kernel workgroups per CU, by (plain,
                                      // candidates, taped), steps per launch and waves per
                                      // block
    int abpc[KMAX_STEPS + 1][17];  // the same for the fused adjoint kernel, by steps
};

static CellArgs cell_args(const lbrs_ctx* c) {
    CellArgs a;
    a.plane = c->plane;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    a.model = c->P.model;
    a.gamma = c->P.gamma;
    a.law = c->P.law;
    for (int k = 0; k < 4; ++k) a.sc[k] = c->P.scalar_flux[k];
    a.code = c->codes;
    if (blocked1d(&c->P)) {
        a.row = BLOCK1D;
        a.fcells = fcells(&c->P);
    }
    return a;
}

static int hip_status(hipError_t e) { return e == hipSuccess ? LBRS_OK : LBRS_E_HIP; }

// Scratch area: the time state, the record of the fused launches, the
// candidate list of the per-step prediction (contexts that can fuse: 2D
// Euler without Dirichlet sides or a body), then the body codes (each at a
// 256-byte boundary).
static size_t round256(size_t n) { return (n + 255) / 256 * 256; }
static size_t pair_offset() { return round256(sizeof(DevState)); }
static size_t cand_offset() { return pair_offset() + round256(sizeof(PairState)); }
static bool fusable(const lbrs_params* p) {
    if (p->model != LBRS_D2Q4 || p->law != LBRS_LAW_EULER || p->solid) return false;
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] == LBRS_BC_DIRICHLET) return false;
    return true;
}
// The time state and the record's step limit, contiguous in the scratch area.
static size_t round_state_bytes() {
    return pair_offset() + offsetof(PairState, n_limit) + sizeof(long long);
}
static size_t codes_offset(const lbrs_params* p) {
    return cand_offset() + (fusable(p) ? round256(sizeof(PredCand) * (size_t)PRED_CAP) : 0);
}

extern "C" {

int lbrs_query_sizes(const lbrs_params* p, size_t* f_bytes, size_t* u_bytes, size_t* scratch_bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    size_t cells = (size_t)p->nx * (size_t)p->ny;
    if (f_bytes) *f_bytes = sizeof(double) * (size_t)nq(p->model) * nk(p) * (size_t)fcells(p);
    if (u_bytes) *u_bytes = sizeof(double) * (size_t)nk(p) * cells;
    if (scratch_bytes)
        *scratch_bytes = codes_offset(p) + (p->solid ? (2 * cells + 255) / 256 * 256 : 0);
    return LBRS_OK;
}

double lbrs_cfl_max(int model) {
    if (model < LBRS_D1Q2 || model > LBRS_D2Q4) return -1.0;
    return cfl_limit(model);
}

int lbrs_body_codes(const lbrs_params* p, unsigned short* h_codes) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!p->solid || !h_codes) return LBRS_E_INVAL;
    return build_body_codes(p, h_codes);
}

int lbrs_prim_to_cons(const lbrs_params* p, const double* d_W, double* d_U, void* hip_stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!d_W || !d_U || d_W == d_U) return LBRS_E_INVAL;
    if (p->law == LBRS_LAW_SCALAR)  // the conserved scalar is the primitive one
        return hip_status(hipMemcpyAsync(d_U, d_W, sizeof(double) * (size_t)p->nx * p->ny,
                                         hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
    CellArgs a;
    a.plane = (long long)p->nx * p->ny;
    a.ps = a.plane;
    a.rs = p->nx;
    a.nx = p->nx;
    a.ny = p->ny;
    a.model = p->model;
    a.gamma = p->gamma;
    return hip_status(launch_prim_to_cons(a, d_W, d_U, (hipStream_t)hip_stream));
}

static CellArgs cell_args_of(const lbrs_params* p) {
    CellArgs a;
    a.plane = (long long)p->nx * p->ny;
    a.ps = a.plane;
    a.rs = p->nx;
    a.nx = p->nx;
    a.ny = p->ny;
    a.model = p->model;
    a.gamma = p->gamma;
    return a;
}

int lbrs_prim_to_cons_adjoint(const lbrs_params* p, const double* d_W, const double* d_Ubar,
                              double* d_Wbar, void* hip_stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!d_W || !d_Ubar || !d_Wbar || d_Wbar == d_W || d_Wbar == d_Ubar) return LBRS_E_INVAL;
    if (p->law != LBRS_LAW_EULER) return LBRS_E_INVAL;
    return hip_status(launch_prim_to_cons_adjoint(cell_args_of(p), d_W, d_Ubar, d_Wbar,
                                                  (hipStream_t)hip_stream));
}

int lbrs_isentropic_to_cons(const lbrs_params* p, const double* d_rho, double* d_U, void* hip_stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!d_rho || !d_U || d_rho == d_U) return LBRS_E_INVAL;
    if (p->law != LBRS_LAW_EULER) return LBRS_E_INVAL;
    return hip_status(launch_isentropic_to_cons(cell_args_of(p), d_rho, d_U, (hipStream_t)hip_stream));
}

int lbrs_isentropic_to_cons_adjoint(const lbrs_params* p, const double* d_rho, const double* d_Ubar,
                                    double* d_rhobar, void* hip_stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!d_rho || !d_Ubar || !d_rhobar || d_rhobar == d_rho || d_rhobar == d_Ubar) return LBRS_E_INVAL;
    if (p->law != LBRS_LAW_EULER) return LBRS_E_INVAL;
    return hip_status(launch_isentropic_to_cons_adjoint(cell_args_of(p), d_rho, d_Ubar, d_rhobar,
                                                        (hipStream_t)hip_stream));
}

// Fill a context and enqueue the initialisation (f^0 = f^eq(U0)); body codes
// need a host staging copy (malloc) and a synchronisation: `allow_body` is
// false for the no-allocation entry point, which rejects bodies.
static int ctx_setup(lbrs_ctx* c, const lbrs_params* p, const double* d_U0, double* d_f0,
                     double* d_f1, void* d_scratch, void* hip_stream, bool allow_body) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!d_U0 || !d_f0 || !d_f1 || !d_scratch || d_f0 == d_f1) return LBRS_E_INVAL;
    if (((uintptr_t)d_scratch & 7u) != 0) return LBRS_E_INVAL;
    if (p->solid && !allow_body) return LBRS_E_INVAL;
    memset(c, 0, sizeof(*c));
    c->P = *p;
    c->Q = nq(p->model);
    c->K = nk(p);
    c->dim = p->model == LBRS_D2Q4 ? 2 : 1;
    c->plane = (long long)p->nx * p->ny;
    if (blocked1d(p)) {
        c->ps = BLOCK1D;
        c->rs = (long long)c->Q * c->K * BLOCK1D;
    } else if (p->layout == LBRS_LAYOUT_ROWS) {
        c->ps = p->nx;
        c->rs = (long long)c->Q * c->K * p->nx;
    } else {
        c->ps = c->plane;
        c->rs = p->nx;
    }
    c->dx = (p->x1 - p->x0) / p->nx;
    c->f0 = d_f0;
    c->f1 = d_f1;
    c->st = (DevState*)d_scratch;
    c->pst = (PairState*)((char*)d_scratch + pair_offset());
    c->cand = fusable(p) ? (PredCand*)((char*)d_scratch + cand_offset()) : nullptr;
    c->fuse = 1;
    c->rounds = true;
    c->stream = (hipStream_t)hip_stream;
    c->launches = 0;
    c->rows_per_tile = 0;
    c->waves_per_block = 4;
    c->alternate = p->solid ? 0 : 1;
    c->dir = false;
    for (int s = 0; s < 4; ++s) c->dir = c->dir || p->bc[s] == LBRS_BC_DIRICHLET;
    c->codes = nullptr;
    c->P.solid = nullptr;  // the host mask is not kept
    if (p->solid) {
        // node codes, built here and copied into the scratch area behind the
        // time state (the copy completes before this call returns)
        const size_t n = (size_t)p->nx * p->ny;
        unsigned short* h = (unsigned short*)malloc(2 * n);
        if (!h) return LBRS_E_NOMEM;
        rc = build_body_codes(p, h);
        if (rc) {
            free(h);
            return rc;
        }
        c->codes = (unsigned short*)((char*)d_scratch + codes_offset(p));
        hipError_t e = hipMemcpyAsync(c->codes, h, 2 * n, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        free(h);
        if (e != hipSuccess) return LBRS_E_HIP;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return LBRS_E_HIP;
    c->persistent_max = persistent1d_max_cells(c->Q, prop.sharedMemPerBlock);
    c->cu_count = prop.multiProcessorCount;
    CellArgs a = cell_args(c);
    const double* dir[4];
    for (int s = 0; s < 4; ++s) dir[s] = p->bc[s] == LBRS_BC_DIRICHLET ? p->dirichlet[s] : nullptr;
    hipError_t e = launch_reset(c->st, c->stream);
    if (e == hipSuccess) e = launch_pair_reset(c->pst, true, c->stream);
    if (e == hipSuccess)
        e = p->law == LBRS_LAW_SCALAR
                ? launch_scalar_init(a, d_U0, d_f0, c->st, p->lambda_mode, p->lambda_user, p->cfl,
                                     dir, c->stream)
                : launch_init(a, d_U0, d_f0, c->st, p->lambda_mode, p->lambda_user, p->cfl, dir,
                              c->stream);
    return e == hipSuccess ? LBRS_OK : LBRS_E_HIP;
}

int lbrs_init(lbrs_ctx** out, const lbrs_params* p, const double* d_U0, double* d_f0, double* d_f1,
              void* d_scratch, void* hip_stream) {
    if (!out) return LBRS_E_INVAL;
    *out = nullptr;
    lbrs_ctx* c = (lbrs_ctx*)calloc(1, sizeof(lbrs_ctx));
    if (!c) return LBRS_E_NOMEM;
    int rc = ctx_setup(c, p, d_U0, d_f0, d_f1, d_scratch, hip_stream, true);
    if (rc) {
        free(c);
        return rc;
    }
    // the rounds of fused PER_STEP calls read the time state and the step
    // limit back through one pinned copy (else two blocking ones)
    if (fusable(p) && p->lambda_mode == LBRS_LAMBDA_PER_STEP &&
        hipHostMalloc(&c->hst, round_state_bytes(), hipHostMallocDefault) != hipSuccess)
        c->hst = nullptr;
    *out = c;
    return LBRS_OK;
}

int lbrs_set_tile(lbrs_ctx* c, int rows_per_tile, int waves_per_block, int alternate) {
    if (!c) return LBRS_E_INVAL;
    if (rows_per_tile != 0 && (rows_per_tile < 1 || rows_per_tile > 65536)) return LBRS_E_INVAL;
    if (!step2d_wpb_supported(waves_per_block)) return LBRS_E_INVAL;
    if (alternate != 0 && alternate != 1) return LBRS_E_INVAL;
    if (alternate && c->codes) return LBRS_E_STATE;  // body kernels march one way
    c->rows_per_tile = rows_per_tile;
    c->waves_per_block = waves_per_block;
    c->alternate = alternate;
    return LBRS_OK;
}

int lbrs_set_fusion(lbrs_ctx* c, int steps_per_launch) {
    if (!c || steps_per_launch < 1 || steps_per_launch > KMAX_STEPS) return LBRS_E_INVAL;
    if (steps_per_launch >= 2 &&
        (c->dim != 2 || c->P.law != LBRS_LAW_EULER || c->dir || c->codes))
        return LBRS_E_STATE;
    c->fuse = steps_per_launch;
    return LBRS_OK;
}

int lbrs_set_stream(lbrs_ctx* c, void* hip_stream) {
    if (!c) return LBRS_E_INVAL;
    c->stream = (hipStream_t)hip_stream;
    return LBRS_OK;
}

// Row segments per strip.  Automatic: as many as make the tiles one balanced
// round of the resident waves (at least 3 rows each: on small grids a step
// is a chain of row latencies, so short segments pay for their two extra
// halo rows); else ceil(ny / rows).
static int blocks_per_cu(const lbrs_ctx* c) {
    lbrs_ctx* m = const_cast<lbrs_ctx*>(c);
    int w = c->waves_per_block;
    int& n = m->bpc[c->alternate][c->dir ? 1 : 0][w];
    if (n == 0) n = step2d_blocks_per_cu(w, c->alternate != 0, c->dir, c->codes != nullptr);
    return n;
}

static int step2d_segments(const lbrs_ctx* c, int nstrips) {
    const int ny = c->P.ny;
    long long nseg;
    if (c->rows_per_tile > 0) {
        nseg = (ny + c->rows_per_tile - 1) / c->rows_per_tile;
    } else {
        long long waves = (long long)c->cu_count * blocks_per_cu(c) * c->waves_per_block;
        nseg = waves / nstrips;
        long long cap = (ny + 2) / 3;  // at least 3 rows per segment
        if (nseg > cap) nseg = cap;
    }
    if (nseg < 1) nseg = 1;
    if (nseg > ny) nseg = ny;
    return (int)nseg;
}

static int step2d_max_blocks(const lbrs_ctx* c) {
    return c->cu_count * blocks_per_cu(c);
}

static Step2DArgs step2d_args(const lbrs_ctx* c, double t_end, double* tape) {
    Step2DArgs a;
    a.f0 = c->f0;
    a.f1 = c->f1;
    a.st = c->st;
    a.tape = tape;
    a.plane = c->plane;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    // strips of at most 62 columns, as many as a multiple of the waves per
    // workgroup, with the columns spread evenly over them
    const int wpb = c->waves_per_block;
    a.nstrips = ((c->P.nx + 61) / 62 + wpb - 1) / wpb * wpb;
    a.strip = (c->P.nx + a.nstrips - 1) / a.nstrips;
    a.nseg = step2d_segments(c, a.nstrips);
    a.ntiles = a.nstrips * a.nseg;
    a.launch = c->launches;
    a.dx = c->dx;
    a.cfl = c->P.cfl;
    a.omega = c->P.omega;
    a.gamma = c->P.gamma;
    a.t_end = t_end;
    a.lam_mode = c->P.lambda_mode == LBRS_LAMBDA_PER_STEP ? LAM_PER_STEP : LAM_FROZEN;
    for (int s = 0; s < 4; ++s) {
        a.bc[s] = c->P.bc[s];
        a.dir[s] = c->P.bc[s] == LBRS_BC_DIRICHLET ? c->P.dirichlet[s] : nullptr;
    }
    a.code = c->codes;
    return a;
}

static int adjoint_k(lbrs_ctx* c, int k, const double* const* tapes, const double* gn,
                     double* g);

// Fused launches of up to k steps: strips of at most 64 - 2k columns (k halo
// lanes on each side), segments of at least 4 rows.  Per-step speeds run
// the fused launches in the form that lists candidates for the predictions
// of the next launch's bounds.  The taped launches of the gradients take two
// steps.
static bool pair_filter(const lbrs_ctx* c) {
    return c->cand && c->P.lambda_mode == LBRS_LAMBDA_PER_STEP;
}



// Waves per workgroup of the fused kernel: 16-wave groups do not fit its
// registers at the occupancy it needs and run as 12; launches of three or
// more steps and the form that lists candidates (more registers) spill in
// 12-wave groups, and run as 8.
static int pair_wpb(const lbrs_ctx* c, bool tape, int kmax) {
    const int cap = (!tape && pair_filter(c)) || kmax >= 3 ? 8 : 12;
    return c->waves_per_block > cap ? cap : c->waves_per_block;
}

static int pair_max_blocks(const lbrs_ctx* c, bool tape, int kmax) {
    lbrs_ctx* m = const_cast<lbrs_ctx*>(c);
    const int w = pair_wpb(c, tape, kmax);
    const int form = tape ? 2 : (pair_filter(c) ? 1 : 0);
    int& n = m->pbpc[form][kmax][w];
    if (n == 0) n = step2d_pair_blocks_per_cu(w, form == 1, kmax, tape);
    return c->cu_count * n;
}

// Launches of up to kmax steps (default: the context's fusion).
static Pair2DArgs pair_args(const lbrs_ctx* c, double t_end, bool tape = false, int kmax = 0) {
    Pair2DArgs a;
    a.f0 = c->f0;
    a.f1 = c->f1;
    a.st = c->st;
    a.pst = c->pst;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    a.kmax = kmax > 0 ? kmax : c->fuse;
    const int wpb = pair_wpb(c, tape, a.kmax);
    const int cols = 64 - 2 * a.kmax;
    a.nstrips = ((c->P.nx + cols - 1) / cols + wpb - 1) / wpb * wpb;
    a.strip = (c->P.nx + a.nstrips - 1) / a.nstrips;
    long long nseg;
    if (c->rows_per_tile > 0) {
        nseg = (c->P.ny + c->rows_per_tile - 1) / c->rows_per_tile;
    } else {
        nseg = (long long)pair_max_blocks(c, tape, a.kmax) * wpb / a.nstrips;
        const long long cap = (c->P.ny + 3) / 4;
        if (nseg > cap) nseg = cap;
    }
    if (nseg < 1) nseg = 1;
    if (nseg > c->P.ny) nseg = c->P.ny;
    a.nseg = (int)nseg;
    a.ntiles = a.nstrips * a.nseg;
    a.launch = c->launches;
    a.dx = c->dx;
    a.cfl = c->P.cfl;
    a.omega = c->P.omega;
    a.gamma = c->P.gamma;
    a.t_end = t_end;
    a.lam_mode = c->P.lambda_mode == LBRS_LAMBDA_PER_STEP ? LAM_PER_STEP : LAM_FROZEN;
    for (int s = 0; s < 4; ++s) a.bc[s] = c->P.bc[s];
    a.last = 0;
    for (int i = 0; i < KMAX_STEPS; ++i) a.tape[i] = nullptr;
    a.plane = c->plane;
    a.cand = pair_filter(c) && !tape ? c->cand : nullptr;
    return a;
}

// Scalar laws: the 2D row-marching tiles use the same strip and segment
// decomposition as the Euler step (no lockstep groups, one march direction).
static int scalar_blocks_per_cu(const lbrs_ctx* c) {
    lbrs_ctx* m = const_cast<lbrs_ctx*>(c);
    int& n = m->sbpc[c->waves_per_block];
    if (n == 0) n = scalar2d_blocks_per_cu(c->waves_per_block);
    return n;
}

static int scalar_max_blocks(const lbrs_ctx* c) { return c->cu_count * scalar_blocks_per_cu(c); }

static ScalarArgs scalar_args(const lbrs_ctx* c, double t_end) {
    ScalarArgs a;
    a.f0 = c->f0;
    a.f1 = c->f1;
    a.st = c->st;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    a.strip = a.nstrips = a.nseg = a.ntiles = 0;
    if (c->dim == 2) {
        const int wpb = c->waves_per_block;
        a.nstrips = ((c->P.nx + 61) / 62 + wpb - 1) / wpb * wpb;
        a.strip = (c->P.nx + a.nstrips - 1) / a.nstrips;
        long long nseg;
        if (c->rows_per_tile > 0) {
            nseg = (c->P.ny + c->rows_per_tile - 1) / c->rows_per_tile;
        } else {
            nseg = (long long)c->cu_count * scalar_blocks_per_cu(c) * wpb / a.nstrips;
            const long long cap = (c->P.ny + 7) / 8;
            if (nseg > cap) nseg = cap;
        }
        if (nseg < 1) nseg = 1;
        if (nseg > c->P.ny) nseg = c->P.ny;
        a.nseg = (int)nseg;
        a.ntiles = a.nstrips * a.nseg;
    }
    a.launch = c->launches;
    a.dx = c->dx;
    a.cfl = c->P.cfl;
    a.omega = c->P.omega;
    a.t_end = t_end;
    a.lam_mode = c->P.lambda_mode == LBRS_LAMBDA_PER_STEP ? LAM_PER_STEP : LAM_FROZEN;
    for (int s = 0; s < 4; ++s) {
        a.bc[s] = c->P.bc[s];
        a.dir[s] = c->P.bc[s] == LBRS_BC_DIRICHLET ? c->P.dirichlet[s] : nullptr;
        a.sc[s] = c->P.scalar_flux[s];
    }
    a.blocked = blocked1d(&c->P) ? 1 : 0;
    return a;
}

static Step1DArgs step1d_args(const lbrs_ctx* c, double t_end, int max_steps) {
    Step1DArgs a;
    a.f0 = c->f0;
    a.f1 = c->f1;
    a.st = c->st;
    a.plane = c->plane;
    a.nx = c->P.nx;
    a.launch = c->launches;
    a.dx = c->dx;
    a.cfl = c->P.cfl;
    a.omega = c->P.omega;
    a.gamma = c->P.gamma;
    a.t_end = t_end;
    a.lam_mode = c->P.lambda_mode == LBRS_LAMBDA_PER_STEP ? LAM_PER_STEP : LAM_FROZEN;
    a.periodic = c->P.bc[0] == LBRS_BC_PERIODIC;
    a.max_steps = max_steps;
    a.blocked = blocked1d(&c->P) ? 1 : 0;
    return a;
}

// One call's worth of fused launches: the set-up kernel (the call stops at
// max_steps more steps) and nl launches, each followed by its prediction
// launches with per-step speeds; the last one leaves an ordinary time state.
static int step_fused(lbrs_ctx* c, int max_steps, double t_end, int nl) {
    Pair2DArgs a = pair_args(c, t_end);
    hipError_t e = launch_pair_prepare(c->pst, c->st, (int)(c->launches & 1), max_steps,
                                       c->stream);
    if (e != hipSuccess) return LBRS_E_HIP;
    const int mb = pair_max_blocks(c, false, a.kmax);
    for (int s = 0; s < nl; ++s) {
        a.launch = c->launches;
        a.last = s == nl - 1;
        e = launch_step2d_pair(a, pair_wpb(c, false, a.kmax), false, mb, c->stream);
        ++c->pair_enq;
        if (e == hipSuccess && a.cand) e = launch_pair_predict(a, c->stream);
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
    }
    return LBRS_OK;
}

int lbrs_step(lbrs_ctx* c, int max_steps, double t_end) {
    if (!c || max_steps < 0 || isnan(t_end)) return LBRS_E_INVAL;
    if (max_steps == 0) return LBRS_OK;
    if (c->P.law == LBRS_LAW_SCALAR) {
        for (int s = 0; s < max_steps; ++s) {
            ScalarArgs a = scalar_args(c, t_end);
            hipError_t e = c->dim == 2
                               ? launch_scalar_step2d(a, c->waves_per_block, scalar_max_blocks(c),
                                                      c->stream)
                               : launch_scalar_step1d(a, c->Q, c->stream);
            if (e != hipSuccess) return LBRS_E_HIP;
            ++c->launches;
        }
        return LBRS_OK;
    }
    if (c->dim == 2 && c->fuse >= 2) {
        // Launches needed.  Per-step speeds: a launch advances at least one
        // step, except a bound-only pass or one whose guess is rejected, and
        // the launch after either of those advances at least two, so
        // max_steps launches always suffice -- but most of them usually find
        // the work done.  So, unless the stream is being captured or the
        // context may not wait (the no-allocation entry point), the call
        // enqueues rounds of about max_steps/kmax launches (each round a
        // call of its own for the steps left; at least three launches, so
        // every round advances) and reads after each how far the run got.
        // Fixed speeds: every launch but the last advances
        // kmax steps (a check that rolls back ends the run with a
        // non-physical state) and the last one at least one.
        const bool per_step = c->P.lambda_mode == LBRS_LAMBDA_PER_STEP;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess) return LBRS_E_HIP;
        if (!per_step || !c->rounds || cs != hipStreamCaptureStatusNone) {
            const int k = c->fuse;
            int nl = per_step ? max_steps : (max_steps + k - 2) / k + 1;
            // A graph replays the launches with the launch numbers they were
            // captured with, and the time state and reductions rotate their
            // slots with the launch number modulo six: a multiple of six
            // launches leaves the slots where the call found them, so every
            // replay continues from the state the last one left.
            if (cs != hipStreamCaptureStatusNone) nl = (nl + 5) / 6 * 6;
            return step_fused(c, max_steps, t_end, nl);
        }
        // at most ROUND_MAX launches a round, so that a call of far more
        // steps than t_end leaves enqueues few launches past the work
        constexpr int ROUND_MAX = 512;
        int left = max_steps;
        while (left > 0) {
            const int want = (left + c->fuse - 1) / c->fuse + 2;
            const int rc = step_fused(c, left, t_end, want < ROUND_MAX ? want : ROUND_MAX);
            if (rc) return rc;
            DevState h;
            long long n_limit = 0;
            if (c->hst) {
                // one copy behind the round's last kernel, then one wait
                if (hipMemcpyAsync(c->hst, c->st, round_state_bytes(), hipMemcpyDeviceToHost,
                                   c->stream) != hipSuccess ||
                    hipStreamSynchronize(c->stream) != hipSuccess)
                    return LBRS_E_HIP;
                memcpy(&h, c->hst, sizeof(DevState));
                memcpy(&n_limit, (const char*)c->hst + pair_offset() + offsetof(PairState, n_limit),
                       sizeof(n_limit));
            } else if (hipStreamSynchronize(c->stream) != hipSuccess ||
                       hipMemcpy(&h, c->st, sizeof(DevState), hipMemcpyDeviceToHost) != hipSuccess ||
                       hipMemcpy(&n_limit, &c->pst->n_limit, sizeof(n_limit),
                                 hipMemcpyDeviceToHost) != hipSuccess) {
                return LBRS_E_HIP;
            }
            const Slot& s = h.s[c->launches & 1];
            if (h.status || !(s.t < t_end) || s.n >= n_limit) break;
            left = (int)(n_limit - s.n);
        }
        return LBRS_OK;
    }
    if (c->dim == 2) {
        for (int s = 0; s < max_steps; ++s) {
            Step2DArgs a = step2d_args(c, t_end, nullptr);
            hipError_t e = launch_step2d(a, c->waves_per_block, false, c->alternate != 0,
                                         c->dir, step2d_max_blocks(c), c->stream);
            if (e != hipSuccess) return LBRS_E_HIP;
            ++c->launches;
        }
        return LBRS_OK;
    }
    if (c->P.nx <= c->persistent_max) {
        Step1DArgs a = step1d_args(c, t_end, max_steps);
        hipError_t e = launch_run1d(a, c->Q, c->stream);
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
        return LBRS_OK;
    }
    for (int s = 0; s < max_steps; ++s) {
        Step1DArgs a = step1d_args(c, t_end, 1);
        hipError_t e = launch_step1d(a, c->Q, c->stream);
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
    }
    return LBRS_OK;
}

int lbrs_step_tape(lbrs_ctx* c, double* d_Utape_n) {
    if (!c || !d_Utape_n) return LBRS_E_INVAL;
    if (c->P.law != LBRS_LAW_EULER) return LBRS_E_STATE;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP) return LBRS_E_STATE;
    if (c->dim != 2 || c->dir || c->codes) return LBRS_E_STATE;  // the tape serves the periodic adjoint
    Step2DArgs a = step2d_args(c, INFINITY, d_Utape_n);
    hipError_t e = launch_step2d(a, c->waves_per_block, true, c->alternate != 0, false,
                                 step2d_max_blocks(c), c->stream);
    if (e != hipSuccess) return LBRS_E_HIP;
    ++c->launches;
    return LBRS_OK;
}

int lbrs_get_state(lbrs_ctx* c, double* t, long long* nsteps, double* lambda, unsigned* status,
                   long long* fail_step) {
    if (!c) return LBRS_E_INVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBRS_E_HIP;
    DevState h;
    if (hipMemcpy(&h, c->st, sizeof(DevState), hipMemcpyDeviceToHost) != hipSuccess) return LBRS_E_HIP;
    const Slot& s = h.s[c->launches & 1];
    if (t) *t = s.t;
    if (nsteps) *nsteps = s.n;
    if (lambda) *lambda = s.lam_used;
    if (status) *status = h.status;
    if (fail_step) *fail_step = h.fail_step == ~0ull ? -1 : (long long)h.fail_step;
    return h.status ? LBRS_E_NONPHYSICAL : LBRS_OK;
}

int lbrs_pair_stats(lbrs_ctx* c, long long* counts, int n) {
    if (!c || !counts || n < 0) return LBRS_E_INVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBRS_E_HIP;
    unsigned long long h[PST_COUNT];
    if (hipMemcpy(h, c->pst->stat, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return LBRS_E_HIP;
    for (int i = 0; i < n; ++i)
        counts[i] = i < PST_COUNT ? (long long)h[i] : i == PST_COUNT ? c->pair_enq : 0;
    return LBRS_OK;
}

int lbrs_moments(lbrs_ctx* c, double* d_U) {
    if (!c || !d_U) return LBRS_E_INVAL;
    CellArgs a = cell_args(c);
    if (c->P.law == LBRS_LAW_SCALAR)
        return hip_status(launch_scalar_moments(a, c->f0, c->f1, c->st, (int)(c->launches & 1), d_U,
                                                c->stream));
    return hip_status(launch_moments(a, c->f0, c->f1, c->st, (int)(c->launches & 1), d_U, c->stream));
}

int lbrs_get_f(lbrs_ctx* c, double* d_f) {
    if (!c || !d_f || d_f == c->f0 || d_f == c->f1) return LBRS_E_INVAL;
    CellArgs a = cell_args(c);
    return hip_status(launch_get_f(a, c->f0, c->f1, c->st, (int)(c->launches & 1), d_f, c->stream));
}

int lbrs_set_f(lbrs_ctx* c, const double* d_f, double t, long long n) {
    if (!c || !d_f || d_f == c->f0 || d_f == c->f1 || !isfinite(t) || n < 0) return LBRS_E_INVAL;
    // the new state becomes launch 0: slot 0, buffer f0, bound in slot 0
    c->launches = 0;
    CellArgs a = cell_args(c);
    hipError_t e = launch_set_f(a, c->f0, c->f1, c->st, d_f, t, n,
                                c->P.lambda_mode == LBRS_LAMBDA_PER_STEP, c->stream);
    // a prediction of the fused launches belonged to the old state
    if (e == hipSuccess) e = launch_pair_reset(c->pst, false, c->stream);
    return hip_status(e);
}

int lbrs_window_objective(lbrs_ctx* c, int ix0, int ix1, int iy0, int iy1, double* d_J,
                          double* d_fbar) {
    if (!c || !d_J || !d_fbar) return LBRS_E_INVAL;
    if (c->dim != 2 || c->P.law != LBRS_LAW_EULER) return LBRS_E_STATE;
    if (ix0 < 0 || iy0 < 0 || ix1 > c->P.nx || iy1 > c->P.ny || ix0 > ix1 || iy0 > iy1)
        return LBRS_E_INVAL;
    CellArgs a = cell_args(c);
    return hip_status(launch_window_objective(a, c->f0, c->f1, c->st, (int)(c->launches & 1), ix0,
                                              ix1, iy0, iy1, d_J, d_fbar, c->stream));
}

int lbrs_adjoint_step(lbrs_ctx* c, const double* d_Utape_n, const double* d_fbar_next, double* d_fbar) {
    if (!c || !d_Utape_n || !d_fbar_next || !d_fbar || d_fbar == d_fbar_next) return LBRS_E_INVAL;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    for (int s = 0; s < 4; ++s)
        if (c->P.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    AdjArgs a;
    a.plane = c->plane;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    a.gamma = c->P.gamma;
    a.omega = c->P.omega;
    a.st = c->st;
    return hip_status(launch_adjoint_step(a, d_Utape_n, d_fbar_next, d_fbar, c->stream));
}

int lbrs_adjoint_step2(lbrs_ctx* c, const double* d_Utape_n1, const double* d_Utape_n,
                       const double* d_fbar_next2, double* d_fbar) {
    if (!c || !d_Utape_n1 || !d_Utape_n || !d_fbar_next2 || !d_fbar || d_fbar == d_fbar_next2)
        return LBRS_E_INVAL;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    for (int s = 0; s < 4; ++s)
        if (c->P.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    const double* tapes[2] = {d_Utape_n1, d_Utape_n};
    return adjoint_k(c, 2, tapes, d_fbar_next2, d_fbar);
}

int lbrs_adjoint_steps(lbrs_ctx* c, int k, const double* d_Utape, const double* d_fbar_next,
                       double* d_fbar) {
    if (!c || !d_Utape || !d_fbar_next || !d_fbar || d_fbar == d_fbar_next || k < 1 ||
        k > KMAX_STEPS)
        return LBRS_E_INVAL;
    if (k == 1) return lbrs_adjoint_step(c, d_Utape, d_fbar_next, d_fbar);
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    for (int s = 0; s < 4; ++s)
        if (c->P.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    const long long ucount = (long long)c->K * c->plane;
    const double* tapes[KMAX_STEPS];
    for (int s = 0; s < k; ++s) tapes[s] = d_Utape + (long long)(k - 1 - s) * ucount;
    return adjoint_k(c, k, tapes, d_fbar_next, d_fbar);
}

int lbrs_adjoint_init(lbrs_ctx* c, const double* d_fbar0, const double* d_U0, double* d_Ubar0) {
    if (!c || !d_fbar0 || !d_U0 || !d_Ubar0) return LBRS_E_INVAL;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    AdjArgs a;
    a.plane = c->plane;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    a.gamma = c->P.gamma;
    a.omega = c->P.omega;
    a.st = c->st;
    return hip_status(launch_adjoint_init(a, d_fbar0, d_U0, d_Ubar0, c->stream));
}

int lbrs_forward_checkpointed(lbrs_ctx* c, int nsteps, int segment, double* d_ckpt) {
    if (!c || !d_ckpt || nsteps < 1 || segment < 1) return LBRS_E_INVAL;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    const long long fcount = (long long)c->Q * c->K * c->plane;
    const int nckpt = (nsteps + segment - 1) / segment;
    for (int j = 0; j < nckpt; ++j) {
        int rc = lbrs_get_f(c, d_ckpt + j * fcount);
        if (rc) return rc;
        int len = nsteps - j * segment < segment ? nsteps - j * segment : segment;
        rc = lbrs_step(c, len, INFINITY);
        if (rc) return rc;
    }
    return LBRS_OK;
}

// k adjoint steps in one launch (k = 2 .. KMAX_STEPS): fbar^{n+k} -> fbar^n
// with tapes[s] = U^{n+k-1-s}, in strips of at most 64 - 2k columns and
// automatic row segments.
static int adjoint_k(lbrs_ctx* c, int k, const double* const* tapes, const double* gn,
                     double* g) {
    AdjPairArgs a;
    a.plane = c->plane;
    a.ps = c->ps;
    a.rs = c->rs;
    a.nx = c->P.nx;
    a.ny = c->P.ny;
    // workgroups of 8 waves at most (12-wave groups spill)
    const int wpb = c->waves_per_block > 8 ? 8 : c->waves_per_block;
    const int cols = 64 - 2 * k;
    a.nstrips = ((c->P.nx + cols - 1) / cols + wpb - 1) / wpb * wpb;
    a.strip = (c->P.nx + a.nstrips - 1) / a.nstrips;
    int& bpc = c->abpc[k][wpb];
    if (bpc == 0) bpc = adjoint_k_blocks_per_cu(wpb, k);
    const int mb = c->cu_count * bpc;
    long long nseg = (long long)mb * wpb / a.nstrips;
    const long long cap = (c->P.ny + 3) / 4;
    if (c->rows_per_tile > 0) nseg = (c->P.ny + c->rows_per_tile - 1) / c->rows_per_tile;
    else if (nseg > cap) nseg = cap;
    if (nseg < 1) nseg = 1;
    if (nseg > c->P.ny) nseg = c->P.ny;
    a.nseg = (int)nseg;
    a.ntiles = a.nstrips * a.nseg;
    a.gamma = c->P.gamma;
    a.omega = c->P.omega;
    a.st = c->st;
    a.k = k;
    for (int s = 0; s < KMAX_STEPS; ++s) a.tape[s] = s < k ? tapes[s] : nullptr;
    a.gn = gn;
    a.g = g;
    return hip_status(launch_adjoint_k(a, wpb, mb, c->stream));
}

// The recompute of a segment in fused launches of up to k = fuse steps
// (fixed lattice speed, so nothing is guessed): every launch but the last
// takes k steps (fewer at the segment's end), launch j steps kj+1 .. kj+k
// writing their input moments to tape slots kj .. kj+k-1, and the last
// launch at most one (a non-physical state ends the run; its tape is not
// used).
static int step_tape_fused(lbrs_ctx* c, int len, double* d_tape) {
    Pair2DArgs a = pair_args(c, INFINITY, true);
    const int k = a.kmax;
    const long long ucount = (long long)c->K * c->plane;
    const int nl = (len + k - 2) / k + 1;
    hipError_t e = launch_pair_prepare(c->pst, c->st, (int)(c->launches & 1), len, c->stream);
    if (e != hipSuccess) return LBRS_E_HIP;
    const int mb = pair_max_blocks(c, true, k);
    for (int j = 0; j < nl; ++j) {
        a.launch = c->launches;
        a.last = j == nl - 1;
        for (int i = 0; i < KMAX_STEPS; ++i) {
            const long long slot = (long long)k * j + i;
            a.tape[i] = d_tape + (slot < len ? slot : len - 1) * ucount;
        }
        e = launch_step2d_pair(a, pair_wpb(c, true, k), true, mb, c->stream);
        ++c->pair_enq;
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
    }
    return LBRS_OK;
}

int lbrs_step_tape2(lbrs_ctx* c, double* d_Utape_n, double* d_Utape_n1) {
    if (!c || !d_Utape_n || !d_Utape_n1 || d_Utape_n == d_Utape_n1) return LBRS_E_INVAL;
    if (c->P.law != LBRS_LAW_EULER) return LBRS_E_STATE;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP) return LBRS_E_STATE;
    if (c->dim != 2 || c->dir || c->codes) return LBRS_E_STATE;
    // the set-up kernel and two launches: the pair, then the one that checks
    // it (a one-step fallback writes slot d_Utape_n, as the first step would)
    Pair2DArgs a = pair_args(c, INFINITY, true, 2);
    hipError_t e = launch_pair_prepare(c->pst, c->st, (int)(c->launches & 1), 2, c->stream);
    if (e != hipSuccess) return LBRS_E_HIP;
    const int mb = pair_max_blocks(c, true, 2);
    a.tape[0] = d_Utape_n;
    a.tape[1] = d_Utape_n1;
    for (int k = 0; k < 2; ++k) {
        a.launch = c->launches;
        a.last = k == 1;
        e = launch_step2d_pair(a, pair_wpb(c, true, 2), true, mb, c->stream);
        ++c->pair_enq;
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
    }
    return LBRS_OK;
}

int lbrs_step_tapes(lbrs_ctx* c, int k, double* d_Utape) {
    if (!c || !d_Utape || k < 1 || k > KMAX_STEPS) return LBRS_E_INVAL;
    if (k == 1) return lbrs_step_tape(c, d_Utape);
    if (c->P.law != LBRS_LAW_EULER) return LBRS_E_STATE;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP) return LBRS_E_STATE;
    if (c->dim != 2 || c->dir || c->codes) return LBRS_E_STATE;
    // the set-up kernel and two launches: the k steps, then the one that
    // checks them (a fallback after a non-physical intermediate state takes
    // the steps up to it, into the same slots)
    Pair2DArgs a = pair_args(c, INFINITY, true, k);
    hipError_t e = launch_pair_prepare(c->pst, c->st, (int)(c->launches & 1), k, c->stream);
    if (e != hipSuccess) return LBRS_E_HIP;
    const int mb = pair_max_blocks(c, true, k);
    const long long ucount = (long long)c->K * c->plane;
    for (int i = 0; i < KMAX_STEPS; ++i) a.tape[i] = d_Utape + (long long)(i < k ? i : k - 1) * ucount;
    for (int j = 0; j < 2; ++j) {
        a.launch = c->launches;
        a.last = j == 1;
        e = launch_step2d_pair(a, pair_wpb(c, true, k), true, mb, c->stream);
        ++c->pair_enq;
        if (e != hipSuccess) return LBRS_E_HIP;
        ++c->launches;
    }
    return LBRS_OK;
}

// Reverse adjoint steps over tape slots len-1 .. 0 (slot i = U^{n0+i}), from
// fbar in cur; cur and nxt swap after every launch, so cur ends holding
// fbar^{n0}.  Fused contexts take up to k = fuse steps per launch (tapes i,
// i-1, .., i-k+1).
static int reverse_sweep(lbrs_ctx* c, int len, const double* d_tape, double*& cur, double*& nxt) {
    const long long ucount = (long long)c->K * c->plane;
    int i = len - 1;
    if (c->fuse >= 2) {
        // launches of fuse steps (tapes i, i-1, ...), then one of the
        // remaining steps (two or more)
        while (i >= 1) {
            const int k = i + 1 < c->fuse ? i + 1 : c->fuse;
            const double* tapes[KMAX_STEPS];
            for (int s = 0; s < k; ++s) tapes[s] = d_tape + (long long)(i - s) * ucount;
            int rc = adjoint_k(c, k, tapes, cur, nxt);
            if (rc) return rc;
            double* t = cur;
            cur = nxt;
            nxt = t;
            i -= k;
        }
    }
    for (; i >= 0; --i) {
        int rc = lbrs_adjoint_step(c, d_tape + i * ucount, cur, nxt);
        if (rc) return rc;
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    return LBRS_OK;
}

int lbrs_backward_checkpointed(lbrs_ctx* c, int nsteps, int segment, const double* d_ckpt,
                               double* d_tape, double* d_fbar, double* d_work) {
    if (!c || !d_ckpt || !d_tape || !d_fbar || !d_work || d_fbar == d_work || nsteps < 1 ||
        segment < 1)
        return LBRS_E_INVAL;
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return LBRS_E_STATE;
    if (c->P.law != LBRS_LAW_EULER || c->codes) return LBRS_E_STATE;
    for (int s = 0; s < 4; ++s)
        if (c->P.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    // time and step count of the first checkpoint (the state the forward
    // sweep started from) and the fixed step size
    DevState h;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBRS_E_HIP;
    if (hipMemcpy(&h, c->st, sizeof(DevState), hipMemcpyDeviceToHost) != hipSuccess) return LBRS_E_HIP;
    const Slot& now = h.s[c->launches & 1];
    const double dt = c->dx / h.lam_fixed;
    const long long n0 = now.n - nsteps;
    const double t0 = now.t - nsteps * dt;
    const long long fcount = (long long)c->Q * c->K * c->plane;
    const long long ucount = (long long)c->K * c->plane;
    const int nckpt = (nsteps + segment - 1) / segment;
    double* cur = d_fbar;
    double* nxt = d_work;
    for (int j = nckpt - 1; j >= 0; --j) {
        int rc = lbrs_set_f(c, d_ckpt + j * fcount, t0 + (double)j * segment * dt, n0 + (long long)j * segment);
        if (rc) return rc;
        int len = nsteps - j * segment < segment ? nsteps - j * segment : segment;
        if (c->fuse >= 2) {
            rc = step_tape_fused(c, len, d_tape);
            if (rc) return rc;
        } else {
            for (int i = 0; i < len; ++i) {
                rc = lbrs_step_tape(c, d_tape + i * ucount);
                if (rc) return rc;
            }
        }
        rc = reverse_sweep(c, len, d_tape, cur, nxt);
        if (rc) return rc;
    }
    if (cur != d_fbar) {
        if (hipMemcpyAsync(d_fbar, cur, sizeof(double) * fcount, hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess)
            return LBRS_E_HIP;
    }
    return LBRS_OK;
}

// The adjoint (fixed-speed, periodic 2D Euler) preconditions of the gradient
// sweeps.
static int gradient_state_ok(const lbrs_ctx* c) {
    if (c->P.lambda_mode == LBRS_LAMBDA_PER_STEP || c->dim != 2) return 0;
    if (c->P.law != LBRS_LAW_EULER || c->codes || c->dir) return 0;
    for (int s = 0; s < 4; ++s)
        if (c->P.bc[s] != LBRS_BC_PERIODIC) return 0;
    return 1;
}

int lbrs_forward_taped(lbrs_ctx* c, int nsteps, double* d_tape) {
    if (!c || !d_tape || nsteps < 1) return LBRS_E_INVAL;
    if (!gradient_state_ok(c)) return LBRS_E_STATE;
    if (c->fuse >= 2) return step_tape_fused(c, nsteps, d_tape);
    const long long ucount = (long long)c->K * c->plane;
    for (int i = 0; i < nsteps; ++i) {
        int rc = lbrs_step_tape(c, d_tape + i * ucount);
        if (rc) return rc;
    }
    return LBRS_OK;
}

int lbrs_backward_taped(lbrs_ctx* c, int nsteps, const double* d_tape, double* d_fbar,
                        double* d_work) {
    if (!c || !d_tape || !d_fbar || !d_work || d_fbar == d_work || nsteps < 1) return LBRS_E_INVAL;
    if (!gradient_state_ok(c)) return LBRS_E_STATE;
    double* cur = d_fbar;
    double* nxt = d_work;
    int rc = reverse_sweep(c, nsteps, d_tape, cur, nxt);
    if (rc) return rc;
    if (cur != d_fbar) {
        const long long fcount = (long long)c->Q * c->K * c->plane;
        if (hipMemcpyAsync(d_fbar, cur, sizeof(double) * fcount, hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess)
            return LBRS_E_HIP;
    }
    return LBRS_OK;
}

// ------------------------------------------------ no-allocation whole run
// The time state of lbrs_run_noalloc lives in this file-scope device array
// (each GPU holds its own copy until the process ends).  Host code never
// passes its name to a kernel: it is a host-side stand-in there.  Its device
// address is looked up once per device, with that device current, and kept.
static constexpr size_t NOALLOC_SCRATCH_BYTES = 512 * 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static constexpr int NOALLOC_MAX_DEVICES = 64;
static void* noalloc_ptr[NOALLOC_MAX_DEVICES];
static int noalloc_state[NOALLOC_MAX_DEVICES];  // 0 unknown, 1 ready, -1 lookup failed

static void* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    int st = __atomic_load_n(&noalloc_state[dev], __ATOMIC_ACQUIRE);
    if (st == 0) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess && ptr) {
            noalloc_ptr[dev] = ptr;  // the same address from every thread that races here
            __atomic_store_n(&noalloc_state[dev], 1, __ATOMIC_RELEASE);
            st = 1;
        } else {
            __atomic_store_n(&noalloc_state[dev], -1, __ATOMIC_RELEASE);
            st = -1;
        }
    }
    return st == 1 ? noalloc_ptr[dev] : nullptr;
}

int lbrs_run_noalloc(const lbrs_params* p, const double* d_U0, double* d_f0, double* d_f1,
                     int max_steps, double t_end, int steps_per_launch, double* d_U,
                     double* d_state, void* hip_stream) {
    if (!p || !d_U || max_steps < 0 || isnan(t_end)) return LBRS_E_INVAL;
    if (steps_per_launch < 1 || steps_per_launch > KMAX_STEPS) return LBRS_E_INVAL;
    if (p->solid) return LBRS_E_INVAL;  // body codes would need a host staging buffer
    // the time state and the fused launches' record must fit the array
    if (codes_offset(p) > NOALLOC_SCRATCH_BYTES) return LBRS_E_INVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LBRS_E_HIP;
    void* sp = noalloc_scratch(dev);
    if (!sp) return LBRS_E_HIP;
    lbrs_ctx c;  // on the stack: nothing is allocated
    int rc = ctx_setup(&c, p, d_U0, d_f0, d_f1, sp, hip_stream, false);
    if (rc) return rc;
    c.rounds = false;  // one enqueue, no waits
    if (steps_per_launch >= 2 && (rc = lbrs_set_fusion(&c, steps_per_launch))) return rc;
    if ((rc = lbrs_step(&c, max_steps, t_end))) return rc;
    if ((rc = lbrs_moments(&c, d_U))) return rc;
    if (d_state &&
        launch_export_state(c.st, (int)(c.launches & 1), d_state, c.stream) != hipSuccess)
        return LBRS_E_HIP;
    return LBRS_OK;
}

const char* lbrs_strerror(int code) {
    switch (code) {
        case LBRS_OK: return "ok";
        case LBRS_E_INVAL: return "invalid argument";
        case LBRS_E_NOMEM: return "host allocation failed";
        case LBRS_E_HIP: return "HIP runtime error";
        case LBRS_E_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
        case LBRS_E_STATE: return "call not valid in this context's mode";
        default: return "unknown error";
    }
}

void lbrs_destroy(lbrs_ctx* c) {
    if (c && c->hst) (void)hipHostFree(c->hst);
    free(c);
}

}  // extern "C"
