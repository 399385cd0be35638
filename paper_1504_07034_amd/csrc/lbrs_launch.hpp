// Launch arguments and launchers shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "lbrs_device.hpp"
#include "lbrs_host.hpp"

namespace lbrs {

struct Step2DArgs {
    double* f0;
    double* f1;
    DevState* st;
    double* tape;         // U^n output [4][ny][nx] (tape kernel only)
    long long plane;      // nx * ny (planes of U and of the tape)
    long long ps, rs;     // population offset = p*ps + y*rs + x
    int nx, ny;
    int strip;            // output columns per strip (<= 62)
    int nstrips, nseg;    // tiles: strips x balanced row segments; nstrips is a
                          // multiple of the waves per workgroup
    int ntiles;
    long long launch;     // host launch counter p
    double dx, cfl, omega, gamma, t_end;
    int lam_mode;
    int bc[4];
    const double* dir[4]; // Dirichlet states per side, [4][n] conserved (or null)
    const unsigned short* code;  // node codes of a solid body [ny][nx] (or null)
};

// Fused launches of up to KMAX_STEPS steps (2D Euler): every step after the
// first takes its lattice speed from the global bound of the state before it,
// which is known only when the launch has ended.  A launch that guesses those
// bounds, or that cannot yet know whether its intermediate states were
// admissible, is tentative: the next launch accepts its result when every
// recorded bound equals its guess bit for bit and every intermediate state
// was admissible; else it falls back to the state before it, now knowing the
// exact bounds up to the first wrong guess, and takes (without guessing) as
// many steps as they allow -- or, where an intermediate state was
// non-physical, exactly the steps up to it, so that the report names the same
// step as single steps would.  The guesses are the predicted bounds when the
// previous launch left them (see PredHeader), else lambda*_n while the bound
// has been repeating (trust > 0); at trust 0 a launch instead reduces the
// bound of f^{n+1} alone (nothing stored) and the next launch steps with it.
// The record lives in slot (p+1) & 1 beside the time state; the intermediate
// states' bounds and flags are slotted like DevState::lam and DevState::bad.
static constexpr int KMAX_STEPS = 4;

struct PairSlot {
    double t_base;              // state before the launch's steps
    long long n_base;
    int cur_base;
    int tentative;              // > 0: the next launch must check this launch's result of
                                // `tentative` steps
    unsigned long long guess[KMAX_STEPS];  // guess[i]: bits of the lambda*_{n+i} taken (i >= 1)
    unsigned long long guess_base;  // bits of lambda*_n of the state before the launch
    int known;                  // 1: this launch only reduced the bound of f^{n+1} (no step)
    int trust;                  // 0..3: +1 when a check finds the bound repeated, -1 when
                                // not; new launches guess while > 0
    int pred_valid;             // predictions left for the state after this launch: pred[i],
    int predicted;              //   i = 1 .. pred_valid, the bound after the next launch's
                                //   i-th step; 1: this launch's guesses were predictions
    unsigned long long pred[KMAX_STEPS];
};

// The prediction of the bounds the next launch needs: after a launch that
// leaves a state S, the launch lists the cells whose bound of S is a local
// maximum (no left, right, lower or upper neighbour's is larger) within
// CAND_REL of the largest its wave has seen and above a floor CAND_REL below
// the bound it guessed or knew for its last step, leaving out the inside of
// flat regions (one cell per wave stands for a region at one value); once
// lambda*(S) is known, a small kernel evaluates the exact bound of the states
// after 1, 2, ... steps from S on the 3 x 3 cells around each candidate (a
// cell's next state pulls from its diagonal neighbours) and takes the
// largest.  Nothing assures that the maximum lies there: a prediction is only
// a guess, which the launch after the next one checks bit for bit like any
// other.
static constexpr double CAND_REL = 1e-4;
// Candidates one launch may leave (more: no prediction).
static constexpr int PRED_CAP = 16384;

// A candidate cell and its bound of U^{n+2}.
struct PredCand {
    long long cell;  // y*nx + x
    double l;
};

// What a fused launch with candidates leaves for the prediction kernel that
// follows it; two of them, by launch parity (a launch fills its own and
// clears the other for the launch after it).
struct PredHeader {
    int armed;                  // 1: the launch listed candidates
    int cur_out;                // buffer holding the state it leaves
    unsigned int ncand;         // candidates written (may exceed PRED_CAP: overflow)
    unsigned int pad;
    double t_out;               // time after the launch's steps
};

// Counters of the fused launches since the context's initialisation.
enum : int {
    PST_PAIRS = 0,        // launches of two or more steps whose result stood
    PST_REJECTED,         // launches of two or more steps rolled back
    PST_BOUND_ONLY,       // launches that only reduced the bound of f^{n+1}
    PST_SINGLE,           // one-step launches
    PST_PREDICTED,        // predictions left for the next launch
    PST_PRED_HIT,         // predicted guesses that stood
    PST_PRED_MISS,        // predicted guesses rolled back
    PST_EVALUATED,        // cells whose bound the prediction kernel evaluated
    PST_PRED_NONE,        // launches with candidates but no prediction (overflow, none)
    PST_LISTED,           // candidates the launches listed
    PST_OVERFLOW,         // launches whose candidates overflowed the list
    PST_STEPS3,           // of PST_PAIRS: three-step launches
    PST_STEPS4,           // of PST_PAIRS: four-step launches
    PST_COUNT
};

struct PairState {
    PairSlot q[2];
    // bounds (bits of doubles >= 0) and non-physical flags of the states
    // after steps 1 .. KMAX_STEPS-1 of a launch; lamk[0] also receives the
    // bound of a bound-only launch
    unsigned long long lamk[KMAX_STEPS - 1][3];
    unsigned int badk[KMAX_STEPS - 1][3];
    unsigned int pad;
    long long n_limit;           // step count at which the current call stops
    PredHeader pred[2];
    unsigned long long stat[PST_COUNT];
};

struct Pair2DArgs {
    double* f0;
    double* f1;
    DevState* st;
    PairState* pst;
    long long ps, rs;     // population offset = p*ps + y*rs + x
    int nx, ny;
    int strip;            // output columns per strip (<= 64 - 2 kmax)
    int nstrips, nseg, ntiles;
    int kmax;             // steps a launch may take (1 .. KMAX_STEPS)
    long long launch;     // host launch counter p
    double dx, cfl, omega, gamma, t_end;
    int lam_mode;
    int bc[4];
    int last;             // last launch of a call: its result must not be tentative
    double* tape[KMAX_STEPS];  // taped form: U^{n+s} of the launch's step s+1 ([4][ny][nx]
                               // each; a launch of k steps writes tape[0 .. k-1])
    long long plane;      // nx * ny
    PredCand* cand;       // candidate list (PRED_CAP entries) of the per-step prediction,
                          // or null: no prediction
};

// 1D population layouts: planar, element (p, x) at p*nx + x, or blocked,
// the planes of each 64-cell block contiguous: (x/64)*QK*64 + p*64 + x%64
// (the last block padded).
__host__ __device__ inline long long ofs1d(bool blocked, long long plane, long long bstride, int p,
                                          long long x) {
    return blocked ? (x >> 6) * bstride + p * BLOCK1D + (x & (BLOCK1D - 1)) : p * plane + x;
}

struct Step1DArgs {
    double* f0;
    double* f1;
    DevState* st;
    long long plane;   // nx
    int nx;
    int blocked;       // blocked 1D layout (block stride Q*3*64)
    long long launch;
    double dx, cfl, omega, gamma, t_end;
    int lam_mode;
    int periodic;
    int max_steps;     // persistent kernel only
};

enum : int { LAW_EULER = 0, LAW_SCALAR = 1 };

struct CellArgs {
    long long plane;   // nx * ny
    long long ps, rs;  // population offset = p*ps + y*rs + x
    int nx, ny;
    int model;         // D1Q2, D1Q3, D2Q4
    double gamma;
    int law = LAW_EULER;                     // LAW_SCALAR: one conserved scalar u
    double sc[4] = {0.0, 0.0, 0.0, 0.0};     // g1 = sc0 u + sc1 u^2/2, g2 = sc2 u + sc3 u^2/2
    const unsigned short* code = nullptr;    // body node codes (solid cells are skipped)
    int row = 0;             // cells per layout row (0: nx; the blocked 1D layout: 64)
    long long fcells = 0;    // cell slots of a population buffer (0: plane; padded when blocked)
};

// Offset of population plane p of cell c (row-major cell index).
__host__ __device__ inline long long cell_ofs(const CellArgs& a, int p, long long c) {
    const int row = a.row > 0 ? a.row : a.nx;
    return p * a.ps + (c / row) * a.rs + c % row;
}

// One step of a scalar law on the D2Q4 lattice (row-marching tiles) or on the
// D1Q2 / D1Q3 lattice (LDS tiles); the time-state protocol is the Euler step's.
struct ScalarArgs {
    double* f0;
    double* f1;
    DevState* st;
    long long ps, rs;       // population offset = p*ps + y*rs + x
    int nx, ny;
    int strip, nstrips, nseg, ntiles;  // 2D tiles, as in Step2DArgs
    long long launch;
    double dx, cfl, omega, t_end;
    int lam_mode;
    int bc[4];
    const double* dir[4];   // prescribed u along Dirichlet sides ([ny] x-sides, [nx] y-sides)
    double sc[4];
    int blocked;            // 1D: blocked layout (rs = Q*64 is the block stride)
};

struct AdjArgs {
    long long plane;
    long long ps, rs;    // population (and adjoint population) layout
    int nx, ny;
    double gamma, omega;
    const DevState* st;  // the fixed lattice speed is read from st->lam_fixed
};

// k adjoint steps per launch (periodic D2Q4): fbar^n from fbar^{n+k}, with
// U^{n+k-1} .. U^n from the tape; tiles as in Pair2DArgs (strips of at most
// 64 - 2k columns).
struct AdjPairArgs {
    long long plane;
    long long ps, rs;       // population layout
    int nx, ny;
    int strip, nstrips, nseg, ntiles;
    double gamma, omega;
    const DevState* st;     // the fixed lattice speed is read from st->lam_fixed
    int k;                  // adjoint steps of the launch (2 .. KMAX_STEPS)
    const double* tape[KMAX_STEPS];  // tape[s] = U^{n+k-1-s} [4][ny][nx], the moments
                                     // step s+1 is taken at
    const double* gn;       // fbar^{n+k}
    double* g;              // fbar^n
};

// team arrival counters sit on separate 128-byte lines
static constexpr int COUNTER_STRIDE = 32;
// largest team (workgroups sharing one unit)
static constexpr int MAXTEAM = 64;

struct Unit1D {
    long long off;     // first cell of the unit in the pools
    int n;             // cells
    int periodic;
    int g;             // members
    int lam_mode;
    double dx, gamma, omega, cfl, t_end, lam_fixed;
};

struct UnitState1D {
    double t;
    long long nsteps;
    double lam_used;
    unsigned status;   // bit 0: non-physical; bit 1: team barrier timed out
    unsigned pad;
    long long fail_step;
};

struct Job1D {
    int unit, member, c0, c1;  // cells [c0, c1) of the unit
};

// Team exchange slot of one member for one step parity.
struct EdgeSlot {
    double lam;
    unsigned bad;
    unsigned pad;
    double first[9];   // f^{n+1} of the member's first cell
    double last[9];    // f^{n+1} of the member's last cell
};

struct Batch1DArgs {
    const Unit1D* units;
    UnitState1D* states;
    const Job1D* jobs;
    const int* job_begin;      // [grid + 1]
    unsigned* counters;        // per unit (stride COUNTER_STRIDE), team barrier arrivals
    EdgeSlot* slots;           // per unit: [2][g] at slot_off[unit]
    const long long* slot_off;
    double* f;                 // pool [Q*3][total]
    long long total;           // pool plane stride
    int Q;
    int max_steps;
    unsigned spin_limit;
};

hipError_t launch_batch1d_init(const Unit1D* units, Unit1D* units_rw, int nunits, const double* U0,
                               double* f, long long total, UnitState1D* states, int Q, hipStream_t s);
hipError_t launch_zero_counters(unsigned* c, int n, hipStream_t s);
hipError_t launch_batch1d(const Batch1DArgs& a, int grid, int threads, int chunk, hipStream_t s);
int batch1d_blocks_per_cu(int Q, int threads, int chunk);
size_t batch1d_lds_bytes(int chunk);

// One domain of a 2D batch (periodic or other sides, fixed lattice speed).
// Its cells are [coff, coff + nx*ny) of the moment pools ([K][total]); its
// populations the block of 16*nx*ny doubles at 16*coff of the population
// pools, row-interleaved ([ny][16][nx]).
struct Domain2D {
    long long coff;
    long long tile0;       // first tile of the domain in the batch's tile list
    long long row0;        // first row of the domain among all domains' rows
    long long ptile0;      // the same in the tile list of the fused launches
    int nx, ny;
    int strip, nstrips, nseg;
    int pstrip, pnstrips;  // strips of the fused launches (<= 64 - 2k columns for k steps)
    int bc[4];
    double dx, gamma, omega, cfl, lam;
    int lam_mode;
    int pad;
};

struct Batch2DArgs {
    const Domain2D* doms;
    int ndom;
    long long ntiles;
    long long pntiles;     // tiles of the fused launches
    long long total;       // cells of all domains
    double* f0;
    double* f1;
    int cur;               // buffer holding f^n (host parity)
    double* tape;          // [4][total] or null
    double* ktape[KMAX_STEPS];  // fused taped launches: U^{n+s} of step s+1 ([4][total])
    unsigned* status;      // per domain
};

hipError_t launch_step2d_batch(const Batch2DArgs& a, int wpb, bool tape, int max_blocks,
                               hipStream_t s);
// k fused steps of every domain (fixed lattice speeds, k = 2 .. KMAX_STEPS;
// the taped form: 2), f^n in buffer a.cur.
hipError_t launch_step2d_batch_pair(const Batch2DArgs& a, int wpb, bool tape, int k,
                                    int max_blocks, hipStream_t s);
int step2d_batch_pair_blocks_per_cu(int wpb, int k);
hipError_t launch_scalar_step2d(const ScalarArgs& a, int wpb, int max_blocks, hipStream_t s);
hipError_t launch_scalar_step1d(const ScalarArgs& a, int q, hipStream_t s);
int scalar2d_blocks_per_cu(int wpb);
hipError_t launch_scalar_init(const CellArgs& a, const double* U0, double* f0, DevState* st,
                              int lam_mode, double lam_user, double cfl,
                              const double* const dir[4], hipStream_t s);
hipError_t launch_scalar_bound_f(const CellArgs& a, const double* f, DevState* st, hipStream_t s);
hipError_t launch_scalar_moments(const CellArgs& a, const double* f0, const double* f1,
                                 const DevState* st, int slot, double* U, hipStream_t s);
// The body kernels (a.code set) march one direction and have no tape.
hipError_t launch_step2d(const Step2DArgs& a, int wpb, bool tape, bool alt, bool dir,
                         int max_blocks, hipStream_t s);
int step2d_blocks_per_cu(int wpb, bool alt, bool dir, bool body = false);
bool step2d_wpb_supported(int wpb);
// Fused launches of up to a.kmax steps (same waves-per-workgroup choices as the step).
hipError_t launch_step2d_pair(const Pair2DArgs& a, int wpb, bool tape, int max_blocks,
                              hipStream_t s);
int step2d_pair_blocks_per_cu(int wpb, bool cand, int kmax, bool tape);
// Start of a call of max_steps fused launches: clears the first-step
// accumulators and records the step count to stop at.
hipError_t launch_pair_prepare(PairState* ps, const DevState* st, int slot, long long max_steps,
                               hipStream_t s);
// After fused launch a.launch: evaluate its candidates and leave the
// predictions (or none) for the next launch (levels 1 .. a.kmax-1).
hipError_t launch_pair_predict(const Pair2DArgs& a, hipStream_t s);
// Clear the fused launches' record (a prediction left for the state, open
// checks) and, with counters, their counters (context initialisation).
hipError_t launch_pair_reset(PairState* ps, bool counters, hipStream_t s);
hipError_t launch_step1d(const Step1DArgs& a, int Q, hipStream_t s);
hipError_t launch_run1d(const Step1DArgs& a, int Q, hipStream_t s);
int persistent1d_max_cells(int Q, size_t lds_limit);
hipError_t launch_reset(DevState* st, hipStream_t s);
hipError_t launch_export_state(const DevState* st, int slot, double* out, hipStream_t s);
hipError_t launch_prim_to_cons(const CellArgs& a, const double* W, double* U, hipStream_t s);
hipError_t launch_prim_to_cons_adjoint(const CellArgs& a, const double* W, const double* Ub,
                                       double* Wb, hipStream_t s);
hipError_t launch_isentropic_to_cons(const CellArgs& a, const double* rho, double* U, hipStream_t s);
hipError_t launch_isentropic_to_cons_adjoint(const CellArgs& a, const double* rho, const double* Ub,
                                             double* rb, hipStream_t s);
hipError_t launch_init(const CellArgs& a, const double* U0, double* f0, DevState* st, int lam_mode,
                       double lam_user, double cfl, const double* const dir[4], hipStream_t s);
hipError_t launch_set_f(const CellArgs& a, double* f0, double* f1, DevState* st, const double* ext,
                        double t, long long n, bool per_step, hipStream_t s);
hipError_t launch_get_f(const CellArgs& a, double* f0, double* f1, const DevState* st, int slot,
                        double* ext, hipStream_t s);
hipError_t launch_moments(const CellArgs& a, const double* f0, const double* f1, const DevState* st,
                          int slot, double* U, hipStream_t s);
hipError_t launch_window_objective(const CellArgs& a, const double* f0, const double* f1,
                                   DevState* st, int slot, int ix0, int ix1, int iy0, int iy1,
                                   double* J, double* fbar, hipStream_t s);
hipError_t launch_pool_moments(const CellArgs& a, const double* f, double* U, hipStream_t s);
hipError_t launch_adjoint_step(const AdjArgs& a, const double* Un, const double* gn, double* g,
                               hipStream_t s);
hipError_t launch_adjoint_init(const AdjArgs& a, const double* fb0, const double* U0, double* Ub,
                               hipStream_t s);
hipError_t launch_adjoint_k(const AdjPairArgs& a, int wpb, int max_blocks, hipStream_t s);
int adjoint_k_blocks_per_cu(int wpb, int k);
// Two adjoint steps of every domain of a 2D batch (tiles of the fused launches).
struct Batch2DAdjPairArgs {
    const Domain2D* doms;
    int ndom;
    long long pntiles;
    long long total;        // cells of all domains (plane of the tapes)
    int k;                  // adjoint steps of the launch (2 .. KMAX_STEPS)
    const double* tape[KMAX_STEPS];  // tape[s] = U^{n+k-1-s} [4][total]
    const double* gn;       // fbar^{n+k}
    double* g;              // fbar^n
};
hipError_t launch_b2_adjoint_k(const Batch2DAdjPairArgs& a, int wpb, int max_blocks,
                               hipStream_t s);
int b2_adjoint_k_blocks_per_cu(int wpb, int k);

}  // namespace lbrs
