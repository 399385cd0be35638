// Host-side checks of the C ABI (declared in lbrs_host.hpp).
#include "lbrs_host.hpp"

#include <math.h>
#include <stdint.h>

namespace lbrs {

int nq(int model) { return model == LBRS_D1Q2 ? 2 : (model == LBRS_D1Q3 ? 3 : 4); }

// Is this the blocked 1D population layout (LAYOUT_ROWS for a 1D model)?
bool blocked1d(const lbrs_params* p) {
    return p->model != LBRS_D2Q4 && p->layout == LBRS_LAYOUT_ROWS;
}
// Cell slots of one population buffer (the blocked 1D layout pads the last block).
long long fcells(const lbrs_params* p) {
    if (blocked1d(p)) return ((long long)p->nx + BLOCK1D - 1) / BLOCK1D * BLOCK1D;
    return (long long)p->nx * p->ny;
}
int nk(const lbrs_params* p) {
    return p->law == LBRS_LAW_SCALAR ? 1 : (p->model == LBRS_D2Q4 ? 4 : 3);
}

int check_params(const lbrs_params* p) {
    if (!p) return LBRS_E_INVAL;
    if (p->model < LBRS_D1Q2 || p->model > LBRS_D2Q4) return LBRS_E_INVAL;
    const int dim = p->model == LBRS_D2Q4 ? 2 : 1;
    if (p->nx < 3 || p->ny < 1) return LBRS_E_INVAL;
    if (dim == 1 && p->ny != 1) return LBRS_E_INVAL;
    if (dim == 2 && p->ny < 3) return LBRS_E_INVAL;
    if ((long long)p->nx * p->ny > (1ll << 40)) return LBRS_E_INVAL;
    if (!(p->x1 > p->x0) || !isfinite(p->x0) || !isfinite(p->x1)) return LBRS_E_INVAL;
    if (p->law != LBRS_LAW_EULER && p->law != LBRS_LAW_SCALAR) return LBRS_E_INVAL;
    if (p->law == LBRS_LAW_EULER && (!(p->gamma > 1.0) || !isfinite(p->gamma))) return LBRS_E_INVAL;
    if (p->law == LBRS_LAW_SCALAR)
        for (int k = 0; k < 4; ++k)
            if (!isfinite(p->scalar_flux[k])) return LBRS_E_INVAL;
    if (!(p->omega > 0.0 && p->omega < 2.0)) return LBRS_E_INVAL;
    if (dim == 2) {
        if (!(p->y1 > p->y0)) return LBRS_E_INVAL;
        double dx = (p->x1 - p->x0) / p->nx, dy = (p->y1 - p->y0) / p->ny;
        if (!(fabs(dx - dy) <= 1e-12 * dx)) return LBRS_E_INVAL;
    }
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] < LBRS_BC_TRANSMISSIVE || p->bc[s] > LBRS_BC_DIRICHLET) return LBRS_E_INVAL;
        if (p->bc[s] == LBRS_BC_DIRICHLET && !p->dirichlet[s]) return LBRS_E_INVAL;
        if (p->bc[s] == LBRS_BC_DIRICHLET && dim != 2 && (p->law == LBRS_LAW_EULER || s >= 2))
            return LBRS_E_INVAL;
        if (p->bc[s] == LBRS_BC_WALL && p->law == LBRS_LAW_SCALAR) return LBRS_E_INVAL;
        if (p->dirichlet[s] && ((uintptr_t)p->dirichlet[s] & 7u) != 0) return LBRS_E_INVAL;
    }
    if ((p->bc[0] == LBRS_BC_PERIODIC) != (p->bc[1] == LBRS_BC_PERIODIC)) return LBRS_E_INVAL;
    if (dim == 2 && (p->bc[2] == LBRS_BC_PERIODIC) != (p->bc[3] == LBRS_BC_PERIODIC))
        return LBRS_E_INVAL;
    if (dim == 1 && (p->bc[0] == LBRS_BC_WALL || p->bc[1] == LBRS_BC_WALL)) return LBRS_E_INVAL;
    if (dim == 2 && !p->solid) {  // wall corners take the body rules
        bool xw = p->bc[0] == LBRS_BC_WALL || p->bc[1] == LBRS_BC_WALL;
        bool yw = p->bc[2] == LBRS_BC_WALL || p->bc[3] == LBRS_BC_WALL;
        if (xw && yw) return LBRS_E_INVAL;
    }
    if (p->solid && (dim != 2 || p->law != LBRS_LAW_EULER)) return LBRS_E_INVAL;
    if (p->lambda_mode < LBRS_LAMBDA_PER_STEP || p->lambda_mode > LBRS_LAMBDA_USER)
        return LBRS_E_INVAL;
    if (p->lambda_mode == LBRS_LAMBDA_USER && !(p->lambda_user > 0.0 && isfinite(p->lambda_user)))
        return LBRS_E_INVAL;
    if (p->lambda_mode != LBRS_LAMBDA_USER && !(p->cfl > 0.0 && p->cfl <= cfl_limit(p->model)))
        return LBRS_E_INVAL;
    if (p->layout != LBRS_LAYOUT_PLANAR && p->layout != LBRS_LAYOUT_ROWS) return LBRS_E_INVAL;
    return LBRS_OK;
}

// The D2Q4 sign patterns in the library's population order.
static const int kSx[4] = {-1, +1, +1, -1};
static const int kSy[4] = {-1, -1, +1, +1};

// Solid test of a position that may lie outside the grid: beyond a WALL side
// always; else the mask at the position wrapped (periodic axis) or clamped.
static bool solid_pos(const lbrs_params* p, int x, int y) {
    const int nx = p->nx, ny = p->ny;
    if (x < 0 && p->bc[0] == LBRS_BC_WALL) return true;
    if (x >= nx && p->bc[1] == LBRS_BC_WALL) return true;
    if (y < 0 && p->bc[2] == LBRS_BC_WALL) return true;
    if (y >= ny && p->bc[3] == LBRS_BC_WALL) return true;
    if (x < 0 || x >= nx)
        x = p->bc[0] == LBRS_BC_PERIODIC ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
    if (y < 0 || y >= ny)
        y = p->bc[2] == LBRS_BC_PERIODIC ? ((y % ny) + ny) % ny : (y < 0 ? 0 : ny - 1);
    return p->solid[(size_t)y * nx + x] != 0;
}

// Node codes (the IMG_* rules of lbrs_host.hpp).  For population i of a fluid
// node whose pull source (x - s_ix, y - s_iy) is solid, the rule follows from
// the source's two axis neighbours (x - s_ix, y) and (x, y - s_iy); the image
// source population must itself be pulled from a non-solid position.
int build_body_codes(const lbrs_params* p, unsigned short* codes) {
    const int nx = p->nx, ny = p->ny;
    bool any_fluid = false;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = (size_t)y * nx + x;
            if (p->solid[c]) {
                codes[c] = (unsigned short)CODE_SOLID;
                continue;
            }
            any_fluid = true;
            unsigned code = 0;
            for (int i = 0; i < 4; ++i) {
                if (!solid_pos(p, x - kSx[i], y - kSy[i])) continue;
                const bool bx = solid_pos(p, x - kSx[i], y);
                const bool by = solid_pos(p, x, y - kSy[i]);
                unsigned rule;
                int j;
                if (bx && by) { rule = IMG_CONCAVE; j = i ^ 2; }
                else if (bx) { rule = IMG_FACE_X; j = i ^ 1; }
                else if (by) { rule = IMG_FACE_Y; j = 3 - i; }
                else { rule = IMG_TIP; j = i ^ 2; }
                if (solid_pos(p, x - kSx[j], y - kSy[j])) return LBRS_E_INVAL;
                code |= rule << (3 * i);
            }
            codes[c] = (unsigned short)code;
        }
    return any_fluid ? LBRS_OK : LBRS_E_INVAL;
}

}  // namespace lbrs
