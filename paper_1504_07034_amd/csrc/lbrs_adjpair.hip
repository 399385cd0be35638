// Two adjoint steps per launch (D2Q4, fixed lattice speed, periodic sides).
//
// One adjoint step (the vector-Jacobian product of one LBRS step, Sec. II.D
// update with a fixed lattice speed) maps fbar^{n+1} to fbar^n:
//   fbar*_i(x) = fbar^{n+1}_i(x + s_i)                       (reverse stream)
//   Ubar(x)    = omega [ sum_i fbar*_i / 4 + (A1^T h_x + A2^T h_y)/(4 lambda) ] at U^n(x)
//   fbar^n_i   = (1 - omega) fbar*_i + Ubar.
// Here a wavefront marches rows of fbar^{n+2}, forms the rows of fbar^{n+1}
// (with U^{n+1} from the tape) and feeds each one straight into the second
// adjoint step (with U^n), so fbar^{n+2} is read and fbar^n written once per
// two steps.  The reverse stream pulls populations 0 (-,-) and 1 (+,-) from
// the row below and populations 2 (+,+) and 3 (-,+) from the row above, one
// lane left or right: a row of the input completes the output row above it
// (with the lower populations kept from two rows before), mirroring the
// forward kernel's pipeline.  Lanes, strips (<= 60 columns, two halo lanes
// on each side) and row segments (two halo rows) are those of the fused
// forward kernel; sides are periodic, so every halo position wraps.
#include "lbrs_launch.hpp"
#include "lbrs_rowops.hpp"

namespace lbrs {

namespace {

__device__ inline void load16(double v[16], const double* __restrict__ f, long long ps, long long rs,
                              int j, int xl) {
    const double* __restrict__ row = f + (long long)j * rs;
#pragma unroll
    for (int p = 0; p < 16; ++p) v[p] = row[p * ps + xl];
}

__device__ inline void load4(double v[4], const double* __restrict__ U, long long plane, int nx,
                             int j, int xl) {
    const double* __restrict__ row = U + (long long)j * nx;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = row[k * plane + xl];
}

// Populations 0 and 1 of a row, moved to the lanes of the row above them
// (fbar*_0(x) = fbar_0(x-1, .), fbar*_1(x) = fbar_1(x+1, .)).
__device__ inline void lower_pulls(const double v[16], double d[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        d[k] = lane_from_left(v[0 * 4 + k]);
        d[4 + k] = lane_from_right(v[1 * 4 + k]);
    }
}

// Populations 2 and 3 of a row, moved to the lanes of the row below them
// (fbar*_2(x) = fbar_2(x+1, .), fbar*_3(x) = fbar_3(x-1, .)).
__device__ inline void upper_pulls(const double v[16], double u[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u[k] = lane_from_right(v[2 * 4 + k]);
        u[4 + k] = lane_from_left(v[3 * 4 + k]);
    }
}

// One domain as the march sees it: fbar^{n+2} in, fbar^n out (population
// offset p*ps + y*rs + x), the tapes U^{n+1} (Ua) and U^n (Ub), element
// (k, y, x) at k*plane + y*nx + x.
struct AdjGeom {
    const double* gn;
    double* g;
    const double* Ua;
    const double* Ub;
    long long ps, rs, plane;
    int nx, ny, strip;
    double gamma, omega, lam;
};

template <int WPB>
__device__ __forceinline__ void march_adjoint_pair(const AdjGeom& a, int strip, int y0, int y1,
                                                   int lane) {
    const double lam = a.lam;
    const int nx = a.nx, ny = a.ny;
    const int row_bytes = nx * 8;
    const int x = strip * a.strip - 2 + lane;
    const int xl = map_index(x, nx, true);
    const bool out_lane = lane >= 2 && lane <= a.strip + 1 && x < nx;
    const int voff = out_lane ? x * 8 : 0x7fffffff;
    // rows [y0-1, y1] of fbar^{n+1}, from rows y0-2 .. y1+1 of fbar^{n+2}
    const int a0 = y0 - 1, b0 = y1 + 1;

    double f[16], nxt[16];
    double PA0[8], PA1[8];  // first step: lower pulls of input rows r-1 and r-2
    double PB0[8], PB1[8];  // second step: lower pulls of fbar^{n+1} rows q-1 and q-2
    double tA[4], tB[4], nA[4], nB[4];
    load16(f, a.gn, a.ps, a.rs, map_index(a0 - 1, ny, true), xl);
    load16(nxt, a.gn, a.ps, a.rs, map_index(a0, ny, true), xl);
    lower_pulls(f, PA0);
#pragma unroll
    for (int p = 0; p < 16; ++p) f[p] = nxt[p];
    // loads for the first iteration: its tape rows, then the next input row
    load4(nA, a.Ua, a.plane, nx, map_index(a0, ny, true), xl);
    load4(nB, a.Ub, a.plane, nx, map_index(a0 - 1, ny, true), xl);
    load16(nxt, a.gn, a.ps, a.rs, map_index(a0 + 1, ny, true), xl);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        PA1[k] = PA0[k];
        PB0[k] = PB1[k] = 0.0;
    }
    lower_pulls(f, PA0);

    for (int r = a0 + 1; r <= b0; ++r) {
        // lockstep with the workgroup's neighbouring strips (equal trip counts)
        if (WPB > 1) __builtin_amdgcn_s_barrier();
#pragma unroll
        for (int p = 0; p < 16; ++p) f[p] = nxt[p];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            tA[k] = nA[k];
            tB[k] = nB[k];
        }
        // the next iteration's tape rows and input row, in flight meanwhile
        load4(nA, a.Ua, a.plane, nx, map_index(r, ny, true), xl);
        load4(nB, a.Ub, a.plane, nx, map_index(r - 1, ny, true), xl);
        load16(nxt, a.gn, a.ps, a.rs, map_index(r + 1, ny, true), xl);

        // first step: row o = r-1 of fbar^{n+1}
        double fb[16], u[8];
        upper_pulls(f, u);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            fb[k] = PA1[k];
            fb[8 + k] = u[k];
            PA1[k] = PA0[k];
        }
        lower_pulls(f, PA0);
        double g1[16];
        adjoint_cell_d2q4(fb, tA, a.gamma, a.omega, lam, g1);

        // second step: row q = o of fbar^{n+1} completes row q-1 of fbar^n
        const int q = r - 1;
        upper_pulls(g1, u);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            fb[k] = PB1[k];
            fb[8 + k] = u[k];
            PB1[k] = PB0[k];
        }
        lower_pulls(g1, PB0);
        double g2[16];
        adjoint_cell_d2q4(fb, tB, a.gamma, a.omega, lam, g2);
        // an output row once q > y0; the store is unconditional (an
        // out-of-range offset is dropped), so no wait covers it
        const bool row_out = q > y0;
        double* orow = a.g + (long long)(row_out ? q - 1 : y0) * a.rs;
        const int vo = row_out ? voff : 0x7fffffff;
#pragma unroll
        for (int p = 0; p < 16; ++p) store_row(orow + p * a.ps, row_bytes, vo, g2[p]);
    }
}

}  // namespace

template <int WPB>
__global__ __launch_bounds__(64 * WPB) void adjoint_pair_d2q4(AdjPairArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    AdjGeom g;
    g.gn = a.gn;
    g.g = a.g;
    g.Ua = a.Ua;
    g.Ub = a.Ub;
    g.ps = a.ps;
    g.rs = a.rs;
    g.plane = a.plane;
    g.nx = a.nx;
    g.ny = a.ny;
    g.strip = a.strip;
    g.gamma = a.gamma;
    g.omega = a.omega;
    g.lam = a.st->lam_fixed;
    const int total_waves = gridDim.x * WPB;
    for (int tile = xcd_remap(blockIdx.x, gridDim.x) * WPB + wave; tile < a.ntiles;
         tile += total_waves) {
        const int strip = tile % a.nstrips;
        const int seg = tile / a.nstrips;
        const int y0 = (int)(((long long)seg * a.ny) / a.nseg);
        const int y1 = (int)(((long long)(seg + 1) * a.ny) / a.nseg);
        march_adjoint_pair<WPB>(g, strip, y0, y1, lane);
    }
}

// The same for every domain of a 2D batch (periodic sides, fixed speeds),
// over the fused launches' tile list (as the fused forward batch kernel).
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void b2_adjoint_pair(Batch2DAdjPairArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long total_waves = (long long)gridDim.x * WPB;
    for (long long tile = (long long)xcd_remap(blockIdx.x, gridDim.x) * WPB + wave;
         tile < a.pntiles; tile += total_waves) {
        int lo = 0, hi = a.ndom - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.doms[mid].ptile0 <= tile) lo = mid;
            else hi = mid - 1;
        }
        const Domain2D& d = a.doms[lo];
        AdjGeom g;
        g.gn = a.gn + 16 * d.coff;
        g.g = a.g + 16 * d.coff;
        g.Ua = a.Ua + d.coff;
        g.Ub = a.Ub + d.coff;
        g.ps = d.nx;
        g.rs = 16LL * d.nx;
        g.plane = a.total;
        g.nx = d.nx;
        g.ny = d.ny;
        g.strip = d.pstrip;
        g.gamma = d.gamma;
        g.omega = d.omega;
        g.lam = d.lam;
        const int local = (int)(tile - d.ptile0);
        const int strip = local % d.pnstrips;
        const int seg = local / d.pnstrips;
        const int y0 = (int)(((long long)seg * d.ny) / d.nseg);
        const int y1 = (int)(((long long)(seg + 1) * d.ny) / d.nseg);
        march_adjoint_pair<WPB>(g, strip, y0, y1, lane);
    }
}

template <int WPB>
static hipError_t launch_adjpair_w(const AdjPairArgs& a, int max_blocks, hipStream_t s) {
    int nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((adjoint_pair_d2q4<WPB>), dim3(nblocks), dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static int adjpair_blocks_w() {
    int n = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adjoint_pair_d2q4<WPB>, 64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

#define LBRS_ADJPAIR_WPB_CASES(X) X(1) X(2) X(4) X(6) X(8) X(12)

hipError_t launch_adjoint_pair(const AdjPairArgs& a, int wpb, int max_blocks, hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_adjpair_w<W>(a, max_blocks, s);
    LBRS_ADJPAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

template <int WPB>
static hipError_t launch_b2adjpair_w(const Batch2DAdjPairArgs& a, int max_blocks, hipStream_t s) {
    long long nblocks = (a.pntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((b2_adjoint_pair<WPB>), dim3((unsigned)nblocks), dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static int b2adjpair_blocks_w() {
    int n = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, b2_adjoint_pair<WPB>, 64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_b2_adjoint_pair(const Batch2DAdjPairArgs& a, int wpb, int max_blocks,
                                  hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_b2adjpair_w<W>(a, max_blocks, s);
    LBRS_ADJPAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int b2_adjoint_pair_blocks_per_cu(int wpb) {
#define LBRS_CASE(W) \
    if (wpb == W) return b2adjpair_blocks_w<W>();
    LBRS_ADJPAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

int adjoint_pair_blocks_per_cu(int wpb) {
#define LBRS_CASE(W) \
    if (wpb == W) return adjpair_blocks_w<W>();
    LBRS_ADJPAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

}  // namespace lbrs
