// Device workspace of the IMEX step (sld_state), shared by the step driver and the server.
#pragma once

#include "sld_internal.h"

struct sld_state_s {
    sld_disc disc = nullptr;
    double* vbar = nullptr;   // [ne][2][N] velocity on the main grid
    double* vfoot = nullptr;  // [ne][2][N] its semi-Lagrangian projection
    double* vsbar = nullptr;  // [2][ne][N] viscous solution, component-major
    double* vs = nullptr;     // [nd][2][Npsi] the intermediate dual velocity v*
    double* b = nullptr;      // [ne][N] right-hand side (viscous, then pressure)
};

// Device bytes of a state's workspace.
inline uint64_t sld_state_bytes(const sld_state_s* st) {
    const uint64_t nm = uint64_t(st->disc->mesh->ne) * st->disc->nphi;
    const uint64_t ndv = uint64_t(st->disc->mesh->nd) * 2 * st->disc->npsi;
    return 8 * (7 * nm + ndv);
}
