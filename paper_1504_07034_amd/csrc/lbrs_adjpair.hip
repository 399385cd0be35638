// Two to four adjoint steps per launch (D2Q4, fixed lattice speed, periodic sides).
//
// One adjoint step (the vector-Jacobian product of one LBRS step, Sec. II.D
// update with a fixed lattice speed) maps fbar^{n+1} to fbar^n:
//   fbar*_i(x) = fbar^{n+1}_i(x + s_i)                       (reverse stream)
//   Ubar(x)    = omega [ sum_i fbar*_i / 4 + (A1^T h_x + A2^T h_y)/(4 lambda) ] at U^n(x)
//   fbar^n_i   = (1 - omega) fbar*_i + Ubar.
// Here a wavefront marches rows of fbar^{n+K}, forms the rows of fbar^{n+K-1}
// (with U^{n+K-1} from the tape) and feeds each one straight into the next
// adjoint step, K times (the last with U^n), so fbar^{n+K} is read and fbar^n
// written once per K steps.  The reverse stream pulls populations 0 (-,-)
// and 1 (+,-) from the row below and populations 2 (+,+) and 3 (-,+) from the
// row above, one lane left or right: a row of a step's input completes the
// output row above it (with the lower populations kept from two rows
// before), mirroring the forward kernel's pipeline.  Lanes, strips (<= 64-2K
// columns, K halo lanes on each side) and row segments (K halo rows) are
// those of the fused forward kernel; sides are periodic, so every halo
// position wraps.
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

// One domain as the march sees it: fbar^{n+K} in, fbar^n out (population
// offset p*ps + y*rs + x), the tapes tape[s] = U^{n+K-1-s} of step s
// (element (k, y, x) at k*plane + y*nx + x).
struct AdjGeom {
    const double* gn;
    double* g;
    const double* tape[KMAX_STEPS];
    long long ps, rs, plane;
    int nx, ny, strip;
    double gamma, omega, lam;
};

// K adjoint steps of rows y0..y1-1 of one strip.  Lane l holds column
// x0 - K + l; step s (0-based) takes row j = r - s of its input at row
// iteration r and completes row j - 1 of its output, valid on lanes
// s+1 .. 62-s; rows y0-K .. y1+K-1 of fbar^{n+K} are read and the pipelines
// start as zeros, which only feed rows that are never used (as in the forward
// march).  LPB: the second row of each step's pipeline lives in the wave's
// LDS area pbl, element k of step s at pbl[(s*8 + k)*64 + lane] (each lane
// its own elements, in program order: no barrier).
template <int WPB, int K, bool LPB>
__device__ __forceinline__ void march_adjoint_k(const AdjGeom& a, int strip, int y0, int y1,
                                                int lane, double* pbl) {
    static_assert(K >= 2 && K <= KMAX_STEPS, "adjoint steps per launch");
    const double lam = a.lam;
    const int nx = a.nx, ny = a.ny;
    const int row_bytes = nx * 8;
    const int x = strip * a.strip - K + lane;
    const int xl = map_index(x, nx, true);
    const bool out_lane = lane >= K && lane <= a.strip + K - 1 && x < nx;
    const int voff = out_lane ? x * 8 : 0x7fffffff;

    double P0[K][8];                // per step: lower pulls of its last input row
    double P1[LPB ? 1 : K][8];      // and of the one before
    double tc[K][4], tn[K][4];      // tape rows of this iteration and the next
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            P0[s][k] = 0.0;
            if (LPB) pbl[(s * 8 + k) * 64 + lane] = 0.0;
            else P1[s][k] = 0.0;
        }
    double nxt[16];
    const int r0 = y0 - K;
    load16(nxt, a.gn, a.ps, a.rs, map_index(r0, ny, true), xl);
#pragma unroll
    for (int s = 0; s < K; ++s) load4(tn[s], a.tape[s], a.plane, nx, map_index(r0 - s - 1, ny, true), xl);

    for (int r = r0; r <= y1 + K - 1; ++r) {
        // lockstep with the workgroup's neighbouring strips (equal trip counts)
        if (WPB > 1) __builtin_amdgcn_s_barrier();
        double in[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) in[p] = nxt[p];
#pragma unroll
        for (int s = 0; s < K; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) tc[s][k] = tn[s][k];
        // the next iteration's input row and tape rows, in flight meanwhile
        load16(nxt, a.gn, a.ps, a.rs, map_index(r + 1, ny, true), xl);
#pragma unroll
        for (int s = 0; s < K; ++s) load4(tn[s], a.tape[s], a.plane, nx, map_index(r - s, ny, true), xl);
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int o = r - s - 1;  // this step's output row
            double fb[16], u[8], lo[8];
            upper_pulls(in, u);
            lower_pulls(in, lo);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (LPB) {
                    double* e = pbl + (s * 8 + k) * 64 + lane;
                    fb[k] = *e;
                    *e = P0[s][k];
                } else {
                    fb[k] = P1[LPB ? 0 : s][k];
                    P1[LPB ? 0 : s][k] = P0[s][k];
                }
                fb[8 + k] = u[k];
                P0[s][k] = lo[k];
            }
            double g[16];
            adjoint_cell_d2q4(fb, tc[s], a.gamma, a.omega, lam, g);
            if (s == K - 1) {
                // an output row of the tile; the store is unconditional (an
                // out-of-range offset is dropped), so no wait covers it
                const bool row_out = o >= y0 && o < y1;
                double* orow = a.g + (long long)(row_out ? o : y0) * a.rs;
                const int vo = row_out ? voff : 0x7fffffff;
#pragma unroll
                for (int p = 0; p < 16; ++p) store_row(orow + p * a.ps, row_bytes, vo, g[p]);
            } else {
#pragma unroll
                for (int p = 0; p < 16; ++p) in[p] = g[p];
            }
        }
    }
}

// Kernels of three or more steps keep the second row of their pipelines in
// LDS (as the forward kernels).
template <int K>
struct AdjPipelineInLds {
    static constexpr bool value = K >= 3;
};

}  // namespace

template <int WPB, int K>
__global__ __launch_bounds__(64 * WPB) void adjoint_k_d2q4(AdjPairArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr bool LPB = AdjPipelineInLds<K>::value;
    __shared__ double pb_lds[LPB ? WPB * K * 8 * 64 : 1];
    double* pbl = pb_lds + (LPB ? wave * K * 8 * 64 : 0);
    AdjGeom g;
    g.gn = a.gn;
    g.g = a.g;
#pragma unroll
    for (int i = 0; i < KMAX_STEPS; ++i) g.tape[i] = a.tape[i];
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
        march_adjoint_k<WPB, K, LPB>(g, strip, y0, y1, lane, pbl);
    }
}

// The same for every domain of a 2D batch (periodic sides, fixed speeds),
// over the fused launches' tile list (as the fused forward batch kernel,
// whose strips fit K steps).
template <int WPB, int K>
__global__ __launch_bounds__(64 * WPB) void b2_adjoint_k(Batch2DAdjPairArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr bool LPB = AdjPipelineInLds<K>::value;
    __shared__ double pb_lds[LPB ? WPB * K * 8 * 64 : 1];
    double* pbl = pb_lds + (LPB ? wave * K * 8 * 64 : 0);
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
#pragma unroll
        for (int i = 0; i < KMAX_STEPS; ++i) g.tape[i] = a.tape[i] ? a.tape[i] + d.coff : nullptr;
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
        march_adjoint_k<WPB, K, LPB>(g, strip, y0, y1, lane, pbl);
    }
}

// Launches of three or more steps run in workgroups of 8 waves at most.
template <int WPB, int K>
static hipError_t launch_adj_wk(const AdjPairArgs& a, int max_blocks, hipStream_t s) {
    int nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((adjoint_k_d2q4<WPB, K>), dim3(nblocks), dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static hipError_t launch_adj_w(const AdjPairArgs& a, int max_blocks, hipStream_t s) {
    if (a.k == 2) return launch_adj_wk<WPB, 2>(a, max_blocks, s);
    if constexpr (WPB <= 8) {
        if (a.k == 3) return launch_adj_wk<WPB, 3>(a, max_blocks, s);
        if (a.k == 4) return launch_adj_wk<WPB, 4>(a, max_blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int WPB, int K>
static int adj_occupancy() {
    int n = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adjoint_k_d2q4<WPB, K>, 64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int WPB>
static int adj_blocks_w(int k) {
    if (k == 2) return adj_occupancy<WPB, 2>();
    if constexpr (WPB <= 8) {
        if (k == 3) return adj_occupancy<WPB, 3>();
        if (k == 4) return adj_occupancy<WPB, 4>();
    }
    return 1;
}

template <int WPB, int K>
static hipError_t launch_b2adj_wk(const Batch2DAdjPairArgs& a, int max_blocks, hipStream_t s) {
    long long nblocks = (a.pntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((b2_adjoint_k<WPB, K>), dim3((unsigned)nblocks), dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static hipError_t launch_b2adj_w(const Batch2DAdjPairArgs& a, int max_blocks, hipStream_t s) {
    if (a.k == 2) return launch_b2adj_wk<WPB, 2>(a, max_blocks, s);
    if constexpr (WPB <= 8) {
        if (a.k == 3) return launch_b2adj_wk<WPB, 3>(a, max_blocks, s);
        if (a.k == 4) return launch_b2adj_wk<WPB, 4>(a, max_blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int WPB, int K>
static int b2adj_occupancy() {
    int n = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, b2_adjoint_k<WPB, K>, 64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int WPB>
static int b2adj_blocks_w(int k) {
    if (k == 2) return b2adj_occupancy<WPB, 2>();
    if constexpr (WPB <= 8) {
        if (k == 3) return b2adj_occupancy<WPB, 3>();
        if (k == 4) return b2adj_occupancy<WPB, 4>();
    }
    return 1;
}

#define LBRS_ADJ_WPB_CASES(X) X(1) X(2) X(4) X(6) X(8) X(12)

hipError_t launch_adjoint_k(const AdjPairArgs& a, int wpb, int max_blocks, hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_adj_w<W>(a, max_blocks, s);
    LBRS_ADJ_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int adjoint_k_blocks_per_cu(int wpb, int k) {
#define LBRS_CASE(W) \
    if (wpb == W) return adj_blocks_w<W>(k);
    LBRS_ADJ_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

hipError_t launch_b2_adjoint_k(const Batch2DAdjPairArgs& a, int wpb, int max_blocks,
                               hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_b2adj_w<W>(a, max_blocks, s);
    LBRS_ADJ_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int b2_adjoint_k_blocks_per_cu(int wpb, int k) {
#define LBRS_CASE(W) \
    if (wpb == W) return b2adj_blocks_w<W>(k);
    LBRS_ADJ_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

}  // namespace lbrs
