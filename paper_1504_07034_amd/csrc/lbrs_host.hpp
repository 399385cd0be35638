// Host-side checks of the C ABI: parameter validation, buffer sizes and the
// node codes of a solid body.  Plain C++ (no HIP), so that the same code is
// built into the library by hipcc and, for the sanitizer test, by g++.
#pragma once

#include <stddef.h>

#include "lbrs.h"

namespace lbrs {

// Node codes of a solid body: per population i (0..3, the D2Q4 order) a
// 3-bit rule in bits 3i..3i+2 for a population whose pull source is solid,
// and the solid-cell bit.
enum : unsigned {
    IMG_PULL = 0u,     // pulled as usual
    IMG_FACE_X = 1u,   // population i^1 (s_x reversed), x-momentum negated
    IMG_FACE_Y = 2u,   // population 3-i (s_y reversed), y-momentum negated
    IMG_CONCAVE = 3u,  // population i^2 (opposite), both momenta negated
    IMG_TIP = 4u,      // population i^2, momenta swapped times -s_ix s_iy
    CODE_SOLID = 0x8000u
};

// Cells per block of the blocked 1D population layout.
static constexpr int BLOCK1D = 64;

// Largest admissible CFL number of a model (lattice speed = lambda*/cfl): the
// equilibria stay monotone in U (Bouchut's condition, Sec. II.D) while every
// eigenvalue of df_i^eq/dU is >= 0 -- D1Q2: 1/2 - mu/(2 lambda), cfl <= 1;
// D1Q3 (Sec. II.C, U/3 -+ G/(2 lambda)): 1/3 - mu/(2 lambda), cfl <= 2/3;
// D2Q4: 1/4 - (s . mu)/(4 lambda) with the Sec. II.D bound, cfl <= 1.
inline double cfl_limit(int model) { return model == LBRS_D1Q3 ? 2.0 / 3.0 : 1.0; }

int nq(int model);                          // populations per cell
bool blocked1d(const lbrs_params* p);       // the blocked 1D layout?
long long fcells(const lbrs_params* p);     // cell slots of a population buffer
int nk(const lbrs_params* p);               // conserved components
int check_params(const lbrs_params* p);     // LBRS_OK or LBRS_E_INVAL
// Node codes of p->solid into codes[nx*ny]; LBRS_E_INVAL for an inadmissible
// mask (an image population that would itself come from a solid position, or
// no fluid cell).
int build_body_codes(const lbrs_params* p, unsigned short* codes);

}  // namespace lbrs
