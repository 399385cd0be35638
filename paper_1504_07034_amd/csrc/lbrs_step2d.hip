// Fused LBRS step for the 2D Euler equations on the D2Q4 lattice (gfx950).
//
// One launch = one time step: moments (eq. "moments_system"), flux and
// equilibria (Sec. II.D), relaxation (1-omega) f + omega f^eq and exact
// hopping along the four diagonals (the multi-dimensional LBRS update of
// Sec. II.D), side conditions (specular wall, Sec. II.E; transmissive and
// periodic sides), and the global wave-speed bound of the next step from the
// freshly streamed populations (Sec. II.D Bouchut bound).
//
// Data: 16 population planes, two buffers; element (p, y, x) at
// p*ps + y*rs + x: planar [i][k][y][x] (ps = nx*ny, rs = nx) or row-interleaved
// [y][i][k][x] (ps = nx, rs = 16*nx), where a row of all 16 planes is one
// contiguous 128*nx-byte block (a wave's row touches 2 pages, not 32).
//
// Work decomposition.  A wavefront owns a strip of S <= 62 output columns and
// marches through a segment of rows (down in even segments, up in odd ones).
// Lane l holds column x0 - 1 + l, so lanes 0 and S + 1 are the strip's halo
// columns, recomputed by both neighbouring strips.
// Each row is read once from HBM: the lane computes U, the flux and the 16
// post-collision values of its column, and the diagonal hops become DPP
// wavefront shifts by one lane (x) plus a two-row register pipeline (y):
//   f1^{n+1}(x, r-1) = f1*(x+1, r)   f2^{n+1}(x, r-1) = f2*(x-1, r)
//   f3^{n+1}(x, r+1) = f3*(x-1, r)   f4^{n+1}(x, r+1) = f4*(x+1, r)
// Marching down, output row r-1 is complete after row r is processed
// (marching up, row r+1), so the new moments
// U^{n+1} and the local bound are formed in registers and reduced (wave max,
// one atomic per wave at most) into the next step's lambda*.
//
// The row loop has no branch around memory instructions: the next row is
// always prefetched (row indices are clamped or wrapped into the grid), and
// rows are written with range-checked buffer stores whose halo lanes carry an
// out-of-range offset, so the hardware drops them.  The wait before a row's
// compute therefore covers only that row's loads, never the previous row's
// stores.  Waves loop over tiles (persistent grid sized to the resident
// waves); tiles are numbered strip-fastest and dealt to XCDs in contiguous
// runs.  The waves of a workgroup own adjacent strips of the same row segment
// and march its rows in lockstep (a bare s_barrier per row, no memory fence),
// so the cache lines two strips share are fetched once, while both waves need
// them.  The host makes the strip count a multiple of the waves per workgroup,
// so every wave of a workgroup runs the same number of rows and tiles.
//
// Solid bodies (BODY kernels).  A 16-bit code per node, built on the host,
// says for each population of the node whether its pull source is solid and
// which same-node specular image replaces it (Sec. II.E free-slip principle;
// faces, concave corners and convex corner tips), and marks solid cells.  The
// images only need the node's own freshly streamed populations, so they are
// a register select after the hops; the code of a row is loaded one row ahead
// of its use, ahead of the next row's populations.  Solid cells are written
// as zeros and left out of lambda* and the admissibility check; their
// collision (a division by zero) only feeds values that the images discard.
// Wall sides are folded into the codes, and BODY kernels march one way.
#include "lbrs_launch.hpp"
#include "lbrs_rowops.hpp"

namespace lbrs {

struct Shifted {
    double s1[4], s2[4], n3[4], n4[4];
};

// The four diagonal hops of post-collision values across lanes.
__device__ inline void shift_row(const double fs[16], Shifted& sh) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sh.s1[k] = lane_from_right(fs[0 * 4 + k]);
        sh.s2[k] = lane_from_left(fs[1 * 4 + k]);
        sh.n3[k] = lane_from_left(fs[2 * 4 + k]);
        sh.n4[k] = lane_from_right(fs[3 * 4 + k]);
    }
}

// Geometry and physics of the domain a tile belongs to.
struct TileGeom {
    const double* fin;
    double* fout;
    double* tape;       // U^n planes (TAPE), element (k, y, x) at k*tape_ps + y*nx + x
    long long tape_ps;
    long long ps, rs;   // population offset p*ps + y*rs + x
    int nx, ny;
    int strip, nstrips, nseg;
    double c4lam, omega, gamma;
    int bc[4];
    const double* dir[4];  // Dirichlet states per side ([4][ny] x-sides, [4][nx] y-sides)
    bool any_dir;
    const unsigned short* code;  // body node codes [ny][nx] (BODY kernels)
};

// How a tile's march sees memory.  Odd row segments are marched through the
// domain mirrored in y: march row j is memory row ny-1-j, population i is
// memory population 3-i (the one with the opposite s_y), and the y-momentum
// changes sign.  The LBRS update commutes with this mirror exactly (every
// operation maps to the same operation on negated operands), so both
// directions produce the same bits, while two neighbouring segments now reach
// the rows they both read at the same time (both at the start or both at the
// end of the launch) and the second read is served by the cache.
struct MarchView {
    long long rbase, rstep;  // element offset of march row j: rbase + j * rstep
    long long ibase, istep;  // offset of plane (i, k): ibase + i * istep + k * ps
    long long tbase, tstep;  // offset of march row j in a moment plane: tbase + j * tstep
    double s2;               // sign of the y-momentum component
    int bc_lo, bc_hi;        // side conditions at march rows 0 and ny-1
    const double* dlo;       // Dirichlet states beyond march row 0 / ny-1 ([4][nx])
    const double* dhi;
    bool mirror;
};

// Dirichlet ghost cells of march row j: the post-collision values of a lane
// whose cell lies beyond a DIRICHLET side are replaced by the equilibria of
// the prescribed state at this step's lattice speed (the y-side decides at a
// corner; the x index along a y-side and the row index along an x-side are
// wrapped or clamped like the grid's own).  Rows and lanes that are not
// ghosts keep their values; without any ghost in the wave nothing happens.
__device__ __forceinline__ void dirichlet_ghosts(const TileGeom& g, const MarchView& m, int j,
                                                 int x, int xl, double gm1, double c4lam,
                                                 double fs[16]) {
    const int nx = g.nx, ny = g.ny;
    const bool grow = (j < 0 && m.bc_lo == BC_DIRICHLET) || (j >= ny && m.bc_hi == BC_DIRICHLET);
    const bool glane = !grow && ((x < 0 && g.bc[0] == BC_DIRICHLET) ||
                                 (x >= nx && g.bc[1] == BC_DIRICHLET));
    if (!grow && !__any(glane)) return;
    double Ug[4] = {1.0, 0.0, 0.0, 1.0};  // placeholder for lanes that keep their values
    if (grow) {
        const double* d = j < 0 ? m.dlo : m.dhi;
#pragma unroll
        for (int k = 0; k < 4; ++k) Ug[k] = d[k * nx + xl];
    } else if (glane) {
        const double* d = x < 0 ? g.dir[0] : g.dir[1];
        const int jj = map_index(j, ny, g.bc[2] == BC_PERIODIC);
        const int row = m.mirror ? ny - 1 - jj : jj;
#pragma unroll
        for (int k = 0; k < 4; ++k) Ug[k] = d[k * ny + row];
    }
    Ug[2] = m.s2 * Ug[2];
    const Euler2 e = euler2(Ug, gm1);
    double fq[16];
    equilibria_d2q4(Ug, e, c4lam, fq);
    const bool ghost = grow || glane;
#pragma unroll
    for (int p = 0; p < 16; ++p) fs[p] = ghost ? fq[p] : fs[p];
}

// Populations of a node whose pull sources are solid, from the node's own
// streamed populations go[i*4+k] by the rules of code cd (a solid cell: all
// zero).  The image sources are never imaged themselves (the host rejects
// bodies where they would be), so the selects may read go as it is updated.
__device__ __forceinline__ void body_images(unsigned cd, double go[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const unsigned r = (cd >> (3 * i)) & 7u;
        const int ix = i ^ 1, iy = 3 - i, io = i ^ 2;
        const double c = (i & 1) ? 1.0 : -1.0;  // -s_ix s_iy
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double fx = (k == 1 ? -1.0 : 1.0) * go[ix * 4 + k];
            const double fy = (k == 2 ? -1.0 : 1.0) * go[iy * 4 + k];
            const double fc = (k == 1 || k == 2 ? -1.0 : 1.0) * go[io * 4 + k];
            const double ft = k == 1 ? c * go[io * 4 + 2] : (k == 2 ? c * go[io * 4 + 1] : go[io * 4 + k]);
            double v = go[i * 4 + k];
            v = r == IMG_FACE_X ? fx : v;
            v = r == IMG_FACE_Y ? fy : v;
            v = r == IMG_CONCAVE ? fc : v;
            v = r == IMG_TIP ? ft : v;
            go[i * 4 + k] = v;
        }
    }
    if (cd & CODE_SOLID) {
#pragma unroll
        for (int p = 0; p < 16; ++p) go[p] = 0.0;
    }
}

// The 16 populations of march row j at column xl (a wave-uniform row base
// plus the lane's column, so that the loads take a scalar base address).
__device__ inline void load_view(double v[16], const double* __restrict__ fin, const MarchView& m,
                                 long long ps, int j, unsigned xl) {
    const double* __restrict__ row = fin + (m.rbase + (long long)j * m.rstep);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double x = (row + (m.ibase + i * m.istep + k * ps))[xl];
            v[i * 4 + k] = k == 2 ? m.s2 * x : x;
        }
}

// Rows y0..y1-1 (march coordinates) of one strip: lanes 1..g.strip are output
// columns, lanes 0 and g.strip+1 its halo columns.  Accumulates the lane's
// bound of the new state and its admissibility.
template <bool TAPE, int WPB, bool DIR, bool BODY>
__device__ __forceinline__ void march_tile(const TileGeom& g, const MarchView& m, int strip, int y0,
                                           int y1, int lane, double& lmax, bool& bad) {
    const int nx = g.nx, ny = g.ny;
    const bool px = g.bc[0] == BC_PERIODIC, py = g.bc[2] == BC_PERIODIC;
    const double* __restrict__ fin = g.fin;
    double* __restrict__ fout = g.fout;
    const long long ps = g.ps;
    const double gm1 = g.gamma - 1.0;
    const double c4lam = g.c4lam, omega = g.omega;
    const int row_bytes = nx * 8;
    const int x = strip * g.strip - 1 + lane;
    const int xl = map_index(x, nx, px);
    const bool out_lane = lane >= 1 && lane <= g.strip && x < nx;
    const int voff = out_lane ? x * 8 : 0x7fffffff;
    const bool wall_xlo = g.bc[0] == BC_WALL && x == 0;
    const bool wall_xhi = g.bc[1] == BC_WALL && x == nx - 1;

    // collision of march row j (populations fr), Dirichlet ghosts, hops
    double U[4];
    Shifted sh;
    auto collide_row = [&](const double (&fr)[16], int j) {
        moments_d2q4(fr, U);
        const Euler2 e = euler2(U, gm1);
        double fs[16];
        collide_d2q4(fr, U, e, c4lam, omega, fs);
        if (DIR) dirichlet_ghosts(g, m, j, x, xl, gm1, c4lam, fs);
        shift_row(fs, sh);
    };

    // prologue: rows y0-1 and y0 fill the two-row pipeline (no output)
    double f[16], nxt[16];
    unsigned ccur = 0, cnext = 0;  // body codes of this and the next output row
    load_view(f, fin, m, ps, map_index(y0 - 1, ny, py), xl);
    load_view(nxt, fin, m, ps, map_index(y0, ny, py), xl);
    if (BODY) ccur = g.code[(long long)y0 * nx + xl];
    collide_row(f, y0 - 1);
    double A3[4], A4[4], B3[4], B4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        A3[k] = sh.n3[k];
        A4[k] = sh.n4[k];
    }
#pragma unroll
    for (int p = 0; p < 16; ++p) f[p] = nxt[p];
    load_view(nxt, fin, m, ps, map_index(y0 + 1, ny, py), xl);
    collide_row(f, y0);
    if (TAPE) {
        double* trow = g.tape + m.tbase + y0 * m.tstep;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            store_row(trow + k * g.tape_ps, row_bytes, voff, k == 2 ? m.s2 * U[k] : U[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        B3[k] = A3[k];
        B4[k] = A4[k];
        A3[k] = sh.n3[k];
        A4[k] = sh.n4[k];
    }

    // main loop: row r completes output row r-1
    for (int r = y0 + 1; r <= y1; ++r) {
        // lockstep with the workgroup's neighbouring strips (same trip
        // count by construction); no fence: nothing is exchanged
        if (WPB > 1) __builtin_amdgcn_s_barrier();
#pragma unroll
        for (int p = 0; p < 16; ++p) f[p] = nxt[p];
        if (BODY) cnext = g.code[(long long)map_index(r, ny, py) * nx + xl];
        load_view(nxt, fin, m, ps, map_index(r + 1, ny, py), xl);
        collide_row(f, r);
        if (TAPE) {
            // U^n of row r; row y1 is the next segment's first row
            double* trow = g.tape + m.tbase + map_index(r, ny, false) * m.tstep;
            const int tv = r < y1 ? voff : 0x7fffffff;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                store_row(trow + k * g.tape_ps, row_bytes, tv, k == 2 ? m.s2 * U[k] : U[k]);
        }
        const int o = r - 1;
        double go[16];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            go[0 * 4 + k] = sh.s1[k];
            go[1 * 4 + k] = sh.s2[k];
            go[2 * 4 + k] = B3[k];
            go[3 * 4 + k] = B4[k];
        }
        // specular reflection at wall node rows/columns: the incoming
        // populations mirror the outgoing ones, normal momentum negated
        // (with a body the codes hold the walls)
        const bool wall_top = !BODY && m.bc_hi == BC_WALL && o == ny - 1;
        const bool wall_bot = !BODY && m.bc_lo == BC_WALL && o == 0;
        bool fluid = true;
        if (BODY) {
            if (__any(ccur != 0)) body_images(ccur, go);
            fluid = (ccur & CODE_SOLID) == 0;
            ccur = cnext;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double sy = (k == 2) ? -1.0 : 1.0, sx = (k == 1) ? -1.0 : 1.0;
            if (wall_top) {
                go[0 * 4 + k] = sy * go[3 * 4 + k];
                go[1 * 4 + k] = sy * go[2 * 4 + k];
            }
            if (wall_bot) {
                go[3 * 4 + k] = sy * go[0 * 4 + k];
                go[2 * 4 + k] = sy * go[1 * 4 + k];
            }
            if (!BODY && wall_xlo) {
                go[1 * 4 + k] = sx * go[0 * 4 + k];
                go[2 * 4 + k] = sx * go[3 * 4 + k];
            }
            if (!BODY && wall_xhi) {
                go[0 * 4 + k] = sx * go[1 * 4 + k];
                go[3 * 4 + k] = sx * go[2 * 4 + k];
            }
        }
        double* orow = fout + m.rbase + (long long)o * m.rstep;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                store_row(orow + m.ibase + i * m.istep + k * ps, row_bytes, voff,
                          k == 2 ? m.s2 * go[i * 4 + k] : go[i * 4 + k]);
        double Un[4], l;
        moments_d2q4(go, Un);
        const bool ok = bound_d2q4(Un, g.gamma, &l);
        bad |= out_lane && fluid && !ok;
        lmax = fmax(lmax, out_lane && fluid ? l : 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            B3[k] = A3[k];
            B4[k] = A4[k];
            A3[k] = sh.n3[k];
            A4[k] = sh.n4[k];
        }
    }
}

// One tile: strip `tile % nstrips` over row segment `tile / nstrips`.  With
// ALT, odd segments are marched through the mirrored view, so that they run
// upwards in memory while even ones run downwards; without it every segment
// runs downwards (the view is then a compile-time identity).
template <bool TAPE, int WPB, bool ALT, bool DIR, bool BODY>
__device__ __forceinline__ void step_tile(const TileGeom& g, int tile, int lane, double& lmax,
                                          bool& bad) {
    const int strip = tile % g.nstrips;
    const int seg = tile / g.nstrips;
    const int ny = g.ny;
    int y0 = (int)(((long long)seg * ny) / g.nseg);
    int y1 = (int)(((long long)(seg + 1) * ny) / g.nseg);
    MarchView m;
    if (ALT && (seg & 1)) {
        const int t = y0;
        y0 = ny - y1;
        y1 = ny - t;
        m.rbase = (long long)(ny - 1) * g.rs;
        m.rstep = -g.rs;
        m.ibase = 12 * g.ps;
        m.istep = -4 * g.ps;
        m.tbase = (long long)(ny - 1) * g.nx;
        m.tstep = -(long long)g.nx;
        m.s2 = -1.0;
        m.bc_lo = g.bc[3];
        m.bc_hi = g.bc[2];
        m.dlo = g.dir[3];
        m.dhi = g.dir[2];
        m.mirror = true;
    } else {
        m.rbase = 0;
        m.rstep = g.rs;
        m.ibase = 0;
        m.istep = 4 * g.ps;
        m.tbase = 0;
        m.tstep = g.nx;
        m.s2 = 1.0;
        m.bc_lo = g.bc[2];
        m.bc_hi = g.bc[3];
        m.dlo = g.dir[2];
        m.dhi = g.dir[3];
        m.mirror = false;
    }
    march_tile<TAPE, WPB, DIR, BODY>(g, m, strip, y0, y1, lane, lmax, bad);
}

template <bool TAPE, int WPB, bool ALT, bool DIR, bool BODY>
__global__ __launch_bounds__(64 * WPB) void step2d_d2q4(Step2DArgs a) {
    static_assert(!BODY || (!ALT && !TAPE), "body kernels march one way, without a tape");
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const StepCtl c = step_control(st, ls, a.lam_mode, a.dx, a.cfl, a.t_end);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_state(st, ls, c);
    if (!c.active) return;

    const int lane = threadIdx.x & 63;
    // wave-uniform, so that tile and row indices (and the store descriptors)
    // live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TileGeom g;
    g.fin = c.cur ? a.f1 : a.f0;
    g.fout = c.cur ? a.f0 : a.f1;
    g.tape = a.tape;
    g.tape_ps = a.plane;
    g.ps = a.ps;
    g.rs = a.rs;
    g.nx = a.nx;
    g.ny = a.ny;
    g.strip = a.strip;
    g.nstrips = a.nstrips;
    g.nseg = a.nseg;
    g.c4lam = 1.0 / (4.0 * c.lam);
    g.omega = a.omega;
    g.gamma = a.gamma;
    g.any_dir = false;
    for (int s = 0; s < 4; ++s) {
        g.bc[s] = a.bc[s];
        g.dir[s] = a.dir[s];
        g.any_dir = g.any_dir || a.bc[s] == BC_DIRICHLET;
    }
    g.code = a.code;
    const int total_waves = gridDim.x * WPB;

    double lmax = 0.0;
    bool bad = false;
    for (int tile = xcd_remap(blockIdx.x, gridDim.x) * WPB + wave; tile < a.ntiles;
         tile += total_waves)
        step_tile<TAPE, WPB, ALT, DIR, BODY>(g, tile, lane, lmax, bad);

    if (a.lam_mode == LAM_PER_STEP) {
        double wm = wave_max(lmax);
        if (lane == 0) publish_max(&st->lam[ls.la], wm);
    }
    if (__any(bad) && lane == 0) publish_bad(st, ls, c.n + 1);
}

// The same step over a batch of independent domains at fixed lattice speeds:
// tiles are numbered domain by domain (each domain's tile count a multiple of
// the waves per workgroup, so a workgroup's waves share a domain and a row
// segment); `cur` selects the buffer holding f^n for every domain.
template <bool TAPE, int WPB>
__global__ __launch_bounds__(64 * WPB) void step2d_batch(Batch2DArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total_waves = gridDim.x * WPB;
    for (long long tile = (long long)xcd_remap(blockIdx.x, gridDim.x) * WPB + wave;
         tile < a.ntiles; tile += total_waves) {
        // domain of the tile (binary search over the first tiles)
        int lo = 0, hi = a.ndom - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (a.doms[mid].tile0 <= tile) lo = mid;
            else hi = mid - 1;
        }
        const Domain2D& d = a.doms[lo];
        TileGeom g;
        const long long fo = 16 * d.coff;
        g.fin = (a.cur ? a.f1 : a.f0) + fo;
        g.fout = (a.cur ? a.f0 : a.f1) + fo;
        g.tape = a.tape ? a.tape + d.coff : nullptr;
        g.tape_ps = a.total;
        g.ps = d.nx;
        g.rs = 16LL * d.nx;
        g.nx = d.nx;
        g.ny = d.ny;
        g.strip = d.strip;
        g.nstrips = d.nstrips;
        g.nseg = d.nseg;
        g.c4lam = 1.0 / (4.0 * d.lam);
        g.omega = d.omega;
        g.gamma = d.gamma;
        for (int s = 0; s < 4; ++s) {
            g.bc[s] = d.bc[s];
            g.dir[s] = nullptr;
        }
        g.any_dir = false;
        g.code = nullptr;
        double lmax = 0.0;
        bool bad = false;
        step_tile<TAPE, WPB, true, false, false>(g, (int)(tile - d.tile0), lane, lmax, bad);
        if (__any(bad) && lane == 0) atomicOr(&a.status[lo], 1u);
    }
}

template <bool TAPE, int WPB, bool ALT, bool DIR, bool BODY>
static hipError_t launch_one(const Step2DArgs& a, int max_blocks, hipStream_t s) {
    int nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((step2d_d2q4<TAPE, WPB, ALT, DIR, BODY>), dim3(nblocks), dim3(64 * WPB), 0,
                       s, a);
    return hipGetLastError();
}

// Kernel for (tape, alternate, dirichlet, body); the moment tape exists for
// the adjoint, which needs periodic sides, so it has no Dirichlet or body
// variant, and body kernels march one way.
template <int W>
static hipError_t launch_w(const Step2DArgs& a, bool tape, bool alt, bool dir, int max_blocks,
                           hipStream_t s) {
    if (a.code) {
        if (tape || alt) return hipErrorInvalidValue;
        return dir ? launch_one<false, W, false, true, true>(a, max_blocks, s)
                   : launch_one<false, W, false, false, true>(a, max_blocks, s);
    }
    if (tape) {
        if (dir) return hipErrorInvalidValue;
        return alt ? launch_one<true, W, true, false, false>(a, max_blocks, s)
                   : launch_one<true, W, false, false, false>(a, max_blocks, s);
    }
    if (dir)
        return alt ? launch_one<false, W, true, true, false>(a, max_blocks, s)
                   : launch_one<false, W, false, true, false>(a, max_blocks, s);
    return alt ? launch_one<false, W, true, false, false>(a, max_blocks, s)
               : launch_one<false, W, false, false, false>(a, max_blocks, s);
}

template <class K>
static int occupancy(K kernel, int threads) {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int W>
static int blocks_w(bool alt, bool dir, bool body) {
    if (body)
        return dir ? occupancy(step2d_d2q4<false, W, false, true, true>, 64 * W)
                   : occupancy(step2d_d2q4<false, W, false, false, true>, 64 * W);
    if (dir)
        return alt ? occupancy(step2d_d2q4<false, W, true, true, false>, 64 * W)
                   : occupancy(step2d_d2q4<false, W, false, true, false>, 64 * W);
    return alt ? occupancy(step2d_d2q4<false, W, true, false, false>, 64 * W)
               : occupancy(step2d_d2q4<false, W, false, false, false>, 64 * W);
}

#define LBRS_WPB_CASES(X) X(1) X(2) X(4) X(6) X(8) X(12) X(16)

hipError_t launch_step2d(const Step2DArgs& a, int wpb, bool tape, bool alt, bool dir,
                         int max_blocks, hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_w<W>(a, tape, alt, dir, max_blocks, s);
    LBRS_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

template <bool TAPE, int WPB>
static hipError_t launch_batch_one(const Batch2DArgs& a, int max_blocks, hipStream_t s) {
    long long nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    hipLaunchKernelGGL((step2d_batch<TAPE, WPB>), dim3((unsigned)nblocks), dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_step2d_batch(const Batch2DArgs& a, int wpb, bool tape, int max_blocks,
                               hipStream_t s) {
#define LBRS_CASE(W)                                                                      \
    if (wpb == W) return tape ? launch_batch_one<true, W>(a, max_blocks, s)              \
                              : launch_batch_one<false, W>(a, max_blocks, s);
    LBRS_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

bool step2d_wpb_supported(int wpb) {
#define LBRS_CASE(W) if (wpb == W) return true;
    LBRS_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return false;
}

// Resident workgroups of the step kernel per CU for a workgroup size.
int step2d_blocks_per_cu(int wpb, bool alt, bool dir, bool body) {
#define LBRS_CASE(W) \
    if (wpb == W) return blocks_w<W>(alt, dir, body);
    LBRS_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

}  // namespace lbrs
