// Batch of independent 2D domains (D2Q4, fixed lattice speeds): the pointwise
// kernels around the batched step (initialisation, moments, the adjoint step
// and initialisation, the window objective) and the C ABI of the batch.  The
// step itself is step2d_batch (lbrs_step2d.hip): one launch advances every
// domain by one step.  All calls are asynchronous; the checkpointed gradient
// of the whole batch can be captured in one hipGraph and replayed.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lbrs.h"
#include "lbrs_launch.hpp"

namespace lbrs {

// Domain of a global cell index (binary search over the first cells).
__device__ inline int domain_of_cell(const Domain2D* doms, int ndom, long long c) {
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (doms[mid].coff <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Domain of a global row index.
__device__ inline int domain_of_row(const Domain2D* doms, int ndom, long long r) {
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (doms[mid].row0 <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// population (p, y, x) of domain d in a pool
__device__ inline long long pofs(const Domain2D& d, int p, int y, int x) {
    return 16 * d.coff + ((long long)y * 16 + p) * d.nx + x;
}

__global__ void b2_zero(unsigned long long* bits, unsigned* status, int ndom) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ndom) {
        bits[i] = 0ull;
        status[i] = 0u;
    }
}

// lambda*(U0) per domain (non-physical U0 flags the domain)
__global__ void b2_bound(const Domain2D* doms, int ndom, long long total, const double* __restrict__ U0,
                         unsigned long long* bits, unsigned* status) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int d = domain_of_cell(doms, ndom, c);
    double U[4], l;
    for (int k = 0; k < 4; ++k) U[k] = U0[k * total + c];
    if (!bound_d2q4(U, doms[d].gamma, &l)) atomicOr(&status[d], 1u);
    publish_max(&bits[d], l);
}

__global__ void b2_lambda(Domain2D* doms, int ndom, const unsigned long long* bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ndom && doms[i].lam_mode != LAM_USER)
        doms[i].lam = __longlong_as_double((long long)bits[i]) / doms[i].cfl;
}

// f^0 = f^eq(U0) at the domain's lattice speed
__global__ void b2_init_eq(const Domain2D* doms, int ndom, long long total,
                           const double* __restrict__ U0, double* __restrict__ f) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int di = domain_of_cell(doms, ndom, c);
    const Domain2D& d = doms[di];
    const long long lc = c - d.coff;
    const int y = (int)(lc / d.nx), x = (int)(lc % d.nx);
    double U[4], z[16], fs[16];
    for (int k = 0; k < 4; ++k) U[k] = U0[k * total + c];
    for (int p = 0; p < 16; ++p) z[p] = 0.0;
    Euler2 e = euler2(U, d.gamma - 1.0);
    collide_d2q4(z, U, e, 1.0 / (4.0 * d.lam), 1.0, fs);
    for (int p = 0; p < 16; ++p) f[pofs(d, p, y, x)] = fs[p];
}

__global__ void b2_moments(const Domain2D* doms, int ndom, long long total,
                           const double* __restrict__ f, double* __restrict__ U) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int di = domain_of_cell(doms, ndom, c);
    const Domain2D& d = doms[di];
    const long long lc = c - d.coff;
    const int y = (int)(lc / d.nx), x = (int)(lc % d.nx);
    double fc[16], Uc[4];
    for (int p = 0; p < 16; ++p) fc[p] = f[pofs(d, p, y, x)];
    moments_d2q4(fc, Uc);
    for (int k = 0; k < 4; ++k) U[k * total + c] = Uc[k];
}

// The adjoint of one fixed-speed step (periodic sides) for every domain; one
// workgroup per (global row, 256-column chunk).
__global__ __launch_bounds__(256) void b2_adjoint_step(const Domain2D* doms, int ndom, long long total,
                                                       int xchunks, const double* __restrict__ Un,
                                                       const double* __restrict__ gn,
                                                       double* __restrict__ g) {
    const long long row = blockIdx.x / xchunks;
    const int xc = blockIdx.x % xchunks;
    const int di = domain_of_row(doms, ndom, row);
    const Domain2D& d = doms[di];
    const int y = (int)(row - d.row0);
    const int x = xc * 256 + threadIdx.x;
    if (x >= d.nx) return;
    const int nx = d.nx, ny = d.ny;
    const int xp = x + 1 < nx ? x + 1 : 0, xm = x > 0 ? x - 1 : nx - 1;
    const int yp = y + 1 < ny ? y + 1 : 0, ym = y > 0 ? y - 1 : ny - 1;
    const int sy[4] = {ym, ym, yp, yp}, sx[4] = {xm, xp, xp, xm};
    double fb[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) fb[i * 4 + k] = gn[pofs(d, i * 4 + k, sy[i], sx[i])];
    const long long c = d.coff + (long long)y * nx + x;
    double U[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) U[k] = Un[k * total + c];
    double out[16];
    adjoint_cell_d2q4(fb, U, d.gamma, d.omega, d.lam, out);
#pragma unroll
    for (int p = 0; p < 16; ++p) g[pofs(d, p, y, x)] = out[p];
}

__global__ void b2_adjoint_init(const Domain2D* doms, int ndom, long long total,
                                const double* __restrict__ fb0, const double* __restrict__ U0,
                                double* __restrict__ Ub) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int di = domain_of_cell(doms, ndom, c);
    const Domain2D& d = doms[di];
    const long long lc = c - d.coff;
    const int y = (int)(lc / d.nx), x = (int)(lc % d.nx);
    double fb[16], U[4], out[4];
    for (int p = 0; p < 16; ++p) fb[p] = fb0[pofs(d, p, y, x)];
    for (int k = 0; k < 4; ++k) U[k] = U0[k * total + c];
    adjoint_init_cell_d2q4(fb, U, d.gamma, d.lam, out);
    for (int k = 0; k < 4; ++k) Ub[k * total + c] = out[k];
}

// J_d = sum over the domain's window of rho^2 (one workgroup per domain,
// fixed order) ...
__global__ __launch_bounds__(1024) void b2_window_sum(const Domain2D* doms, const int* win,
                                                      const double* __restrict__ f, double* J) {
    __shared__ double part[16];
    const Domain2D& d = doms[blockIdx.x];
    const int ix0 = win[4 * blockIdx.x], ix1 = win[4 * blockIdx.x + 1];
    const int iy0 = win[4 * blockIdx.x + 2], iy1 = win[4 * blockIdx.x + 3];
    const long long w = ix1 - ix0, cells = w * (long long)(iy1 - iy0);
    double acc = 0.0;
    for (long long j = threadIdx.x; j < cells; j += blockDim.x) {
        const int y = (int)(iy0 + j / w), x = (int)(ix0 + j % w);
        double rho = (f[pofs(d, 0, y, x)] + f[pofs(d, 8, y, x)]) +
                     (f[pofs(d, 4, y, x)] + f[pofs(d, 12, y, x)]);
        acc += rho * rho;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
        J[blockIdx.x] = t;
    }
}

// ... and its seed dJ_d/df_{i,rho} = 2 rho inside the window
__global__ void b2_window_seed(const Domain2D* doms, int ndom, long long total, const int* win,
                               const double* __restrict__ f, double* __restrict__ fbar) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    const int di = domain_of_cell(doms, ndom, c);
    const Domain2D& d = doms[di];
    const long long lc = c - d.coff;
    const int y = (int)(lc / d.nx), x = (int)(lc % d.nx);
    const bool in = x >= win[4 * di] && x < win[4 * di + 1] && y >= win[4 * di + 2] && y < win[4 * di + 3];
    double rho = (f[pofs(d, 0, y, x)] + f[pofs(d, 8, y, x)]) + (f[pofs(d, 4, y, x)] + f[pofs(d, 12, y, x)]);
    for (int p = 0; p < 16; ++p) fbar[pofs(d, p, y, x)] = (in && (p % 4) == 0) ? 2.0 * rho : 0.0;
}

}  // namespace lbrs

using namespace lbrs;

struct lbrs_batch2d {
    int ndom;
    long long total, rows, ntiles;
    int max_nx;
    std::vector<Domain2D> doms;
    std::vector<long long> coff;
    Domain2D* d_doms;
    unsigned long long* d_bits;
    unsigned* d_status;
    int* d_win;
    double* f0;
    double* f1;
    int cur;
    long long nsteps;
    hipStream_t stream;
    int wpb, max_blocks;
    int fuse;                 // time steps per forward launch (1, or 2 to KMAX_STEPS fused)
    long long pntiles;        // tiles of the fused launches
    int pmax_blocks[KMAX_STEPS + 1];  // resident workgroups of the k-step fused kernel
    int amax_blocks[KMAX_STEPS + 1];  // resident workgroups of the k-step adjoint kernel
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void* graph_args[7];  // arguments the captured gradient graph was built with
    long long graph_steps[2];
    int graph_fuse;
    int graph_cur;            // host state (buffer of f^n, step count) at the end of the
    long long graph_nsteps;   // captured sequence, restored after every replay
};

namespace {

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// The tile list of the fused launches of up to k steps (k >= 2): strips of at
// most 64 - 2k columns, a multiple of the waves per workgroup per domain, the
// domain's row segments (host copy; the caller uploads it).
void b2_fused_tiles(lbrs_batch2d* b, int k) {
    const int cols = 64 - 2 * (k < 2 ? 2 : k);
    long long ptiles = 0;
    for (Domain2D& d : b->doms) {
        d.ptile0 = ptiles;
        d.pnstrips = ((d.nx + cols - 1) / cols + b->wpb - 1) / b->wpb * b->wpb;
        d.pstrip = (d.nx + d.pnstrips - 1) / d.pnstrips;
        ptiles += (long long)d.pnstrips * d.nseg;
    }
    b->pntiles = ptiles;
}

static inline unsigned grid_cells(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int b2_check(const lbrs_params* p) {
    if (p->model != LBRS_D2Q4 || p->law != LBRS_LAW_EULER || p->solid || p->nx < 3 || p->ny < 3)
        return LBRS_E_INVAL;
    if (!(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->gamma > 1.0)) return LBRS_E_INVAL;
    if (!(p->omega > 0.0 && p->omega < 2.0)) return LBRS_E_INVAL;
    double dx = (p->x1 - p->x0) / p->nx, dy = (p->y1 - p->y0) / p->ny;
    if (!(fabs(dx - dy) <= 1e-12 * dx)) return LBRS_E_INVAL;
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] < 0 || p->bc[s] > 2) return LBRS_E_INVAL;
    if ((p->bc[0] == 1) != (p->bc[1] == 1) || (p->bc[2] == 1) != (p->bc[3] == 1)) return LBRS_E_INVAL;
    bool xw = p->bc[0] == 2 || p->bc[1] == 2, yw = p->bc[2] == 2 || p->bc[3] == 2;
    if (xw && yw) return LBRS_E_INVAL;
    if (p->lambda_mode == LBRS_LAMBDA_PER_STEP) return LBRS_E_INVAL;  // fixed speeds only
    if (p->lambda_mode == LBRS_LAMBDA_USER && !(p->lambda_user > 0.0)) return LBRS_E_INVAL;
    if (p->lambda_mode == LBRS_LAMBDA_FROZEN_INIT && !(p->cfl > 0.0 && p->cfl <= 1.0)) return LBRS_E_INVAL;
    return LBRS_OK;
}

size_t b2_scratch(int ndom) {
    return al256(sizeof(Domain2D) * ndom) + al256(sizeof(unsigned long long) * ndom) +
           al256(sizeof(unsigned) * ndom) + al256(sizeof(int) * 4 * ndom);
}

bool ok(hipError_t e) { return e == hipSuccess; }

}  // namespace

extern "C" {

int lbrs_batch2d_query(int ndom, const lbrs_params* doms, long long* cell_offsets,
                       size_t* scratch_bytes) {
    if (ndom < 1 || !doms) return LBRS_E_INVAL;
    long long off = 0;
    for (int d = 0; d < ndom; ++d) {
        int rc = b2_check(&doms[d]);
        if (rc) return rc;
        if (cell_offsets) cell_offsets[d] = off;
        off += (long long)doms[d].nx * doms[d].ny;
    }
    if (cell_offsets) cell_offsets[ndom] = off;
    if (scratch_bytes) *scratch_bytes = b2_scratch(ndom);
    return LBRS_OK;
}

int lbrs_batch2d_init(lbrs_batch2d** out, int ndom, const lbrs_params* doms, const double* d_U0,
                      double* d_f0, double* d_f1, void* d_scratch, void* hip_stream) {
    if (!out) return LBRS_E_INVAL;
    *out = nullptr;
    int rc = lbrs_batch2d_query(ndom, doms, nullptr, nullptr);
    if (rc) return rc;
    if (!d_U0 || !d_f0 || !d_f1 || d_f0 == d_f1 || !d_scratch || ((uintptr_t)d_scratch & 255u))
        return LBRS_E_INVAL;
    lbrs_batch2d* b = new (std::nothrow) lbrs_batch2d();
    if (!b) return LBRS_E_NOMEM;
    int dev = 0;
    hipDeviceProp_t prop;
    if (!ok(hipGetDevice(&dev)) || !ok(hipGetDeviceProperties(&prop, dev))) {
        delete b;
        return LBRS_E_HIP;
    }
    b->ndom = ndom;
    b->wpb = 8;
    b->max_blocks = prop.multiProcessorCount * step2d_blocks_per_cu(b->wpb, true, false);
    for (int k = 2; k <= KMAX_STEPS; ++k)
        b->pmax_blocks[k] = prop.multiProcessorCount * step2d_batch_pair_blocks_per_cu(b->wpb, k);
    for (int k = 2; k <= KMAX_STEPS; ++k)
        b->amax_blocks[k] = prop.multiProcessorCount * b2_adjoint_k_blocks_per_cu(b->wpb, k);
    b->fuse = 1;
    b->doms.resize(ndom);
    long long off = 0, rows = 0, tiles = 0;
    b->max_nx = 0;
    for (int i = 0; i < ndom; ++i) {
        const lbrs_params* p = &doms[i];
        Domain2D& d = b->doms[i];
        d.coff = off;
        d.row0 = rows;
        d.tile0 = tiles;
        d.nx = p->nx;
        d.ny = p->ny;
        d.nstrips = ((p->nx + 61) / 62 + b->wpb - 1) / b->wpb * b->wpb;
        d.strip = (p->nx + d.nstrips - 1) / d.nstrips;
        // row segments of about 64 rows (the batch has many tiles per round)
        long long nseg = (p->ny + 63) / 64;
        d.nseg = (int)std::max(1LL, std::min<long long>(nseg, p->ny));
        for (int s = 0; s < 4; ++s) d.bc[s] = p->bc[s];
        d.dx = (p->x1 - p->x0) / p->nx;
        d.gamma = p->gamma;
        d.omega = p->omega;
        d.cfl = p->cfl;
        d.lam_mode = p->lambda_mode == LBRS_LAMBDA_USER ? LAM_USER : LAM_FROZEN;
        d.lam = p->lambda_user;
        d.pad = 0;
        off += (long long)p->nx * p->ny;
        rows += p->ny;
        tiles += (long long)d.nstrips * d.nseg;
        b->max_nx = std::max(b->max_nx, p->nx);
    }
    b->total = off;
    b->rows = rows;
    b->ntiles = tiles;
    b2_fused_tiles(b, 2);
    char* s = (char*)d_scratch;
    b->d_doms = (Domain2D*)s;
    s += al256(sizeof(Domain2D) * ndom);
    b->d_bits = (unsigned long long*)s;
    s += al256(sizeof(unsigned long long) * ndom);
    b->d_status = (unsigned*)s;
    s += al256(sizeof(unsigned) * ndom);
    b->d_win = (int*)s;
    b->f0 = d_f0;
    b->f1 = d_f1;
    b->cur = 0;
    b->nsteps = 0;
    b->stream = (hipStream_t)hip_stream;
    b->graph = nullptr;
    b->exec = nullptr;
    for (auto& a : b->graph_args) a = nullptr;
    b->graph_steps[0] = b->graph_steps[1] = 0;
    bool good = ok(hipMemcpyAsync(b->d_doms, b->doms.data(), sizeof(Domain2D) * ndom,
                                  hipMemcpyHostToDevice, b->stream)) &&
                ok(hipStreamSynchronize(b->stream));
    if (!good) {
        delete b;
        return LBRS_E_HIP;
    }
    *out = b;
    return lbrs_batch2d_reset(b, d_U0);
}

int lbrs_batch2d_reset(lbrs_batch2d* b, const double* d_U0) {
    if (!b || !d_U0) return LBRS_E_INVAL;
    hipStream_t s = b->stream;
    hipLaunchKernelGGL(b2_zero, dim3(grid_cells(b->ndom, 256)), dim3(256), 0, s, b->d_bits, b->d_status,
                       b->ndom);
    hipLaunchKernelGGL(b2_bound, dim3(grid_cells(b->total, 256)), dim3(256), 0, s, b->d_doms, b->ndom,
                       b->total, d_U0, b->d_bits, b->d_status);
    hipLaunchKernelGGL(b2_lambda, dim3(grid_cells(b->ndom, 256)), dim3(256), 0, s, b->d_doms, b->ndom,
                       b->d_bits);
    hipLaunchKernelGGL(b2_init_eq, dim3(grid_cells(b->total, 256)), dim3(256), 0, s, b->d_doms, b->ndom,
                       b->total, d_U0, b->f0);
    b->cur = 0;
    b->nsteps = 0;
    return ok(hipGetLastError()) ? LBRS_OK : LBRS_E_HIP;
}

static Batch2DArgs b2_args(const lbrs_batch2d* b, double* tape) {
    Batch2DArgs a;
    a.doms = b->d_doms;
    a.ndom = b->ndom;
    a.ntiles = b->ntiles;
    a.pntiles = b->pntiles;
    a.total = b->total;
    a.f0 = b->f0;
    a.f1 = b->f1;
    a.cur = b->cur;
    a.tape = tape;
    for (int i = 0; i < KMAX_STEPS; ++i) a.ktape[i] = nullptr;
    a.status = b->d_status;
    return a;
}

int lbrs_batch2d_set_fusion(lbrs_batch2d* b, int steps_per_launch) {
    if (!b || steps_per_launch < 1 || steps_per_launch > KMAX_STEPS) return LBRS_E_INVAL;
    if (steps_per_launch != b->fuse) {
        // the fused launches' strips for this many steps (every fused
        // kernel, the taped and adjoint ones too, walks this tile list),
        // into the device table (whose lattice speeds the device computed)
        const size_t bytes = sizeof(Domain2D) * b->ndom;
        if (!ok(hipStreamSynchronize(b->stream)) ||
            !ok(hipMemcpy(b->doms.data(), b->d_doms, bytes, hipMemcpyDeviceToHost)))
            return LBRS_E_HIP;
        b2_fused_tiles(b, steps_per_launch);
        if (!ok(hipMemcpyAsync(b->d_doms, b->doms.data(), bytes, hipMemcpyHostToDevice,
                               b->stream)) ||
            !ok(hipStreamSynchronize(b->stream)))
            return LBRS_E_HIP;
    }
    b->fuse = steps_per_launch;
    return LBRS_OK;
}

int lbrs_batch2d_step(lbrs_batch2d* b, int nsteps) {
    if (!b || nsteps < 0) return LBRS_E_INVAL;
    if (b->fuse >= 2) {
        // launches of fuse steps, then one of the remaining steps (two or more)
        while (nsteps >= 2) {
            const int k = nsteps < b->fuse ? nsteps : b->fuse;
            if (!ok(launch_step2d_batch_pair(b2_args(b, nullptr), b->wpb, false, k,
                                             b->pmax_blocks[k], b->stream)))
                return LBRS_E_HIP;
            b->cur ^= 1;
            b->nsteps += k;
            nsteps -= k;
        }
    }
    for (int i = 0; i < nsteps; ++i) {
        if (!ok(launch_step2d_batch(b2_args(b, nullptr), b->wpb, false, b->max_blocks, b->stream)))
            return LBRS_E_HIP;
        b->cur ^= 1;
        ++b->nsteps;
    }
    return LBRS_OK;
}

int lbrs_batch2d_step_tape(lbrs_batch2d* b, double* d_Utape) {
    if (!b || !d_Utape) return LBRS_E_INVAL;
    if (!ok(launch_step2d_batch(b2_args(b, d_Utape), b->wpb, true, b->max_blocks, b->stream)))
        return LBRS_E_HIP;
    b->cur ^= 1;
    ++b->nsteps;
    return LBRS_OK;
}

int lbrs_batch2d_moments(lbrs_batch2d* b, double* d_U) {
    if (!b || !d_U) return LBRS_E_INVAL;
    hipLaunchKernelGGL(b2_moments, dim3(grid_cells(b->total, 256)), dim3(256), 0, b->stream, b->d_doms,
                       b->ndom, b->total, b->cur ? b->f1 : b->f0, d_U);
    return ok(hipGetLastError()) ? LBRS_OK : LBRS_E_HIP;
}

int lbrs_batch2d_get_f(lbrs_batch2d* b, double* d_f) {
    if (!b || !d_f) return LBRS_E_INVAL;
    return ok(hipMemcpyAsync(d_f, b->cur ? b->f1 : b->f0, sizeof(double) * 16 * b->total,
                             hipMemcpyDeviceToDevice, b->stream))
               ? LBRS_OK
               : LBRS_E_HIP;
}

int lbrs_batch2d_set_f(lbrs_batch2d* b, const double* d_f, long long n) {
    if (!b || !d_f || n < 0) return LBRS_E_INVAL;
    if (!ok(hipMemcpyAsync(b->f0, d_f, sizeof(double) * 16 * b->total, hipMemcpyDeviceToDevice,
                           b->stream)))
        return LBRS_E_HIP;
    b->cur = 0;
    b->nsteps = n;
    return LBRS_OK;
}

int lbrs_batch2d_adjoint_step(lbrs_batch2d* b, const double* d_Utape, const double* d_fbar_next,
                              double* d_fbar) {
    if (!b || !d_Utape || !d_fbar_next || !d_fbar || d_fbar == d_fbar_next) return LBRS_E_INVAL;
    for (const Domain2D& d : b->doms)
        for (int s = 0; s < 4; ++s)
            if (d.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    const int xchunks = (b->max_nx + 255) / 256;
    hipLaunchKernelGGL(b2_adjoint_step, dim3((unsigned)(b->rows * xchunks)), dim3(256), 0, b->stream,
                       b->d_doms, b->ndom, b->total, xchunks, d_Utape, d_fbar_next, d_fbar);
    return ok(hipGetLastError()) ? LBRS_OK : LBRS_E_HIP;
}

int lbrs_batch2d_adjoint_init(lbrs_batch2d* b, const double* d_fbar0, const double* d_U0,
                              double* d_Ubar0) {
    if (!b || !d_fbar0 || !d_U0 || !d_Ubar0) return LBRS_E_INVAL;
    hipLaunchKernelGGL(b2_adjoint_init, dim3(grid_cells(b->total, 256)), dim3(256), 0, b->stream,
                       b->d_doms, b->ndom, b->total, d_fbar0, d_U0, d_Ubar0);
    return ok(hipGetLastError()) ? LBRS_OK : LBRS_E_HIP;
}

int lbrs_batch2d_set_window(lbrs_batch2d* b, double lo, double hi) {
    if (!b || !(hi >= lo)) return LBRS_E_INVAL;
    std::vector<int> w(4 * b->ndom);
    for (int i = 0; i < b->ndom; ++i) {
        const Domain2D& d = b->doms[i];
        // cells whose centres lie in the closed [lo, hi] on each axis (domain
        // origin at 0; dx = dy)
        int i0 = -1, i1 = -1, j0 = -1, j1 = -1;
        for (int x = 0; x < d.nx; ++x) {
            double c = (x + 0.5) * d.dx;
            if (c >= lo && c <= hi) {
                if (i0 < 0) i0 = x;
                i1 = x + 1;
            }
        }
        for (int y = 0; y < d.ny; ++y) {
            double c = (y + 0.5) * d.dx;
            if (c >= lo && c <= hi) {
                if (j0 < 0) j0 = y;
                j1 = y + 1;
            }
        }
        if (i0 < 0 || j0 < 0) return LBRS_E_INVAL;
        w[4 * i] = i0;
        w[4 * i + 1] = i1;
        w[4 * i + 2] = j0;
        w[4 * i + 3] = j1;
    }
    if (!ok(hipMemcpyAsync(b->d_win, w.data(), sizeof(int) * 4 * b->ndom, hipMemcpyHostToDevice,
                           b->stream)) ||
        !ok(hipStreamSynchronize(b->stream)))
        return LBRS_E_HIP;
    return LBRS_OK;
}

int lbrs_batch2d_window_objective(lbrs_batch2d* b, double* d_J, double* d_fbar) {
    if (!b || !d_J || !d_fbar) return LBRS_E_INVAL;
    const double* f = b->cur ? b->f1 : b->f0;
    hipLaunchKernelGGL(b2_window_sum, dim3(b->ndom), dim3(1024), 0, b->stream, b->d_doms, b->d_win, f, d_J);
    hipLaunchKernelGGL(b2_window_seed, dim3(grid_cells(b->total, 256)), dim3(256), 0, b->stream,
                       b->d_doms, b->ndom, b->total, b->d_win, f, d_fbar);
    return ok(hipGetLastError()) ? LBRS_OK : LBRS_E_HIP;
}

// Whole gradient of J_d (each domain's window objective) with respect to U0:
// reset from U0, forward with checkpoints every `segment` steps, objective,
// k adjoint steps of every domain (fused launch, k <= the fusion the tile
// list was planned for): fbar^{n+k} -> fbar^n with tapes[s] = U^{n+k-1-s}.
static int b2_adjoint_k_step(lbrs_batch2d* b, int k, const double* const* tapes,
                             const double* gn, double* g) {
    Batch2DAdjPairArgs a;
    a.doms = b->d_doms;
    a.ndom = b->ndom;
    a.pntiles = b->pntiles;
    a.total = b->total;
    a.k = k;
    for (int s = 0; s < KMAX_STEPS; ++s) a.tape[s] = s < k ? tapes[s] : nullptr;
    a.gn = gn;
    a.g = g;
    return ok(launch_b2_adjoint_k(a, b->wpb, b->amax_blocks[k], b->stream)) ? LBRS_OK
                                                                            : LBRS_E_HIP;
}

// backward sweep (recompute each segment with a tape, reverse adjoint steps),
// adjoint of the initialisation.  Enqueue only (no host synchronisation).
static int b2_gradient_enqueue(lbrs_batch2d* b, const double* d_U0, int nsteps, int segment,
                               double* d_ckpt, double* d_tape, double* d_fbar, double* d_work,
                               double* d_J, double* d_Ubar0) {
    for (const Domain2D& d : b->doms)  // the adjoint steps are written for periodic sides
        for (int s = 0; s < 4; ++s)
            if (d.bc[s] != LBRS_BC_PERIODIC) return LBRS_E_STATE;
    int rc = lbrs_batch2d_reset(b, d_U0);
    if (rc) return rc;
    const long long fcount = 16 * b->total, ucount = 4 * b->total;
    double* cur = d_fbar;
    double* nxt = d_work;
    // len steps from the current state, U^{n+i} to tape slot i
    auto taped_steps = [&](int len) -> int {
        int i = 0;
        if (b->fuse >= 2) {
            // launches of fuse steps, every step's input taped, then one of
            // the remaining steps (two or more)
            while (i + 1 < len) {
                const int k = len - i < b->fuse ? len - i : b->fuse;
                Batch2DArgs a = b2_args(b, nullptr);
                for (int s = 0; s < k; ++s) a.ktape[s] = d_tape + (long long)(i + s) * ucount;
                if (!ok(launch_step2d_batch_pair(a, b->wpb, true, k, b->pmax_blocks[k],
                                                 b->stream)))
                    return LBRS_E_HIP;
                b->cur ^= 1;
                b->nsteps += k;
                i += k;
            }
        }
        for (; i < len; ++i) {
            int r = lbrs_batch2d_step_tape(b, d_tape + i * ucount);
            if (r) return r;
        }
        return LBRS_OK;
    };
    // adjoint steps back through tape slots len-1 .. 0 (cur and nxt swap)
    auto reverse_steps = [&](int len) -> int {
        int i = len - 1;
        if (b->fuse >= 2) {
            // launches of fuse adjoint steps (tapes i, i-1, ...), then one of
            // the remaining steps (two or more)
            while (i >= 1) {
                const int k = i + 1 < b->fuse ? i + 1 : b->fuse;
                const double* tapes[KMAX_STEPS];
                for (int s = 0; s < k; ++s) tapes[s] = d_tape + (long long)(i - s) * ucount;
                int r = b2_adjoint_k_step(b, k, tapes, cur, nxt);
                if (r) return r;
                std::swap(cur, nxt);
                i -= k;
            }
        }
        for (; i >= 0; --i) {
            int r = lbrs_batch2d_adjoint_step(b, d_tape + i * ucount, cur, nxt);
            if (r) return r;
            std::swap(cur, nxt);
        }
        return LBRS_OK;
    };
    if (segment >= nsteps) {
        // one segment: the forward sweep itself writes the tape of every
        // step, then the adjoint runs straight back (no checkpoint, no
        // recompute; d_ckpt is not used)
        if ((rc = taped_steps(nsteps))) return rc;
        if ((rc = lbrs_batch2d_window_objective(b, d_J, d_fbar))) return rc;
        if ((rc = reverse_steps(nsteps))) return rc;
        return lbrs_batch2d_adjoint_init(b, cur, d_U0, d_Ubar0);
    }
    const int nck = (nsteps + segment - 1) / segment;
    for (int j = 0; j < nck; ++j) {
        if ((rc = lbrs_batch2d_get_f(b, d_ckpt + j * fcount))) return rc;
        int len = std::min(segment, nsteps - j * segment);
        if ((rc = lbrs_batch2d_step(b, len))) return rc;
    }
    if ((rc = lbrs_batch2d_window_objective(b, d_J, d_fbar))) return rc;
    for (int j = nck - 1; j >= 0; --j) {
        if ((rc = lbrs_batch2d_set_f(b, d_ckpt + j * fcount, (long long)j * segment))) return rc;
        int len = std::min(segment, nsteps - j * segment);
        if ((rc = taped_steps(len))) return rc;
        if ((rc = reverse_steps(len))) return rc;
    }
    return lbrs_batch2d_adjoint_init(b, cur, d_U0, d_Ubar0);
}

int lbrs_batch2d_gradient(lbrs_batch2d* b, const double* d_U0, int nsteps, int segment,
                          double* d_ckpt, double* d_tape, double* d_fbar, double* d_work,
                          double* d_J, double* d_Ubar0, int use_graph) {
    if (!b || !d_U0 || !d_ckpt || !d_tape || !d_fbar || !d_work || !d_J || !d_Ubar0 || nsteps < 1 ||
        segment < 1 || d_fbar == d_work)
        return LBRS_E_INVAL;
    if (!use_graph)
        return b2_gradient_enqueue(b, d_U0, nsteps, segment, d_ckpt, d_tape, d_fbar, d_work, d_J, d_Ubar0);
    const void* args[7] = {d_U0, d_ckpt, d_tape, d_fbar, d_work, d_J, d_Ubar0};
    bool same = b->exec && b->graph_steps[0] == nsteps && b->graph_steps[1] == segment &&
                b->graph_fuse == b->fuse;
    for (int i = 0; same && i < 7; ++i) same = b->graph_args[i] == args[i];
    if (b->exec && !same) {  // other arguments: capture a new graph
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    if (!b->exec) {
        hipStream_t cap;
        if (!ok(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking))) return LBRS_E_HIP;
        hipStream_t keep = b->stream;
        b->stream = cap;
        int rc = LBRS_E_HIP;
        hipGraph_t g = nullptr;
        if (ok(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)))
            rc = b2_gradient_enqueue(b, d_U0, nsteps, segment, d_ckpt, d_tape, d_fbar, d_work, d_J, d_Ubar0);
        bool ended = ok(hipStreamEndCapture(cap, &g));
        b->stream = keep;
        (void)hipStreamDestroy(cap);
        if (rc || !ended || !ok(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0))) {
            if (g) (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return rc ? rc : LBRS_E_HIP;
        }
        b->graph = g;
        for (int i = 0; i < 7; ++i) b->graph_args[i] = args[i];
        b->graph_steps[0] = nsteps;
        b->graph_steps[1] = segment;
        b->graph_fuse = b->fuse;
        // enqueueing the sequence advanced the host's view of the state
        // (which buffer holds f^n, the step count) to its end
        b->graph_cur = b->cur;
        b->graph_nsteps = b->nsteps;
    }
    if (!ok(hipGraphLaunch(b->exec, b->stream))) return LBRS_E_HIP;
    // a replay leaves the state where the captured sequence ends, whatever
    // eager calls ran in between
    b->cur = b->graph_cur;
    b->nsteps = b->graph_nsteps;
    return LBRS_OK;
}

int lbrs_batch2d_get_state(lbrs_batch2d* b, long long* nsteps, double* lambda, unsigned* status) {
    if (!b) return LBRS_E_INVAL;
    if (!ok(hipStreamSynchronize(b->stream))) return LBRS_E_HIP;
    std::vector<Domain2D> d(b->ndom);
    std::vector<unsigned> st(b->ndom);
    if (!ok(hipMemcpy(d.data(), b->d_doms, sizeof(Domain2D) * b->ndom, hipMemcpyDeviceToHost)) ||
        !ok(hipMemcpy(st.data(), b->d_status, sizeof(unsigned) * b->ndom, hipMemcpyDeviceToHost)))
        return LBRS_E_HIP;
    if (nsteps) *nsteps = b->nsteps;
    int rc = LBRS_OK;
    for (int i = 0; i < b->ndom; ++i) {
        if (lambda) lambda[i] = d[i].lam;
        if (status) status[i] = st[i];
        if (st[i]) rc = LBRS_E_NONPHYSICAL;
    }
    return rc;
}

void lbrs_batch2d_destroy(lbrs_batch2d* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"
