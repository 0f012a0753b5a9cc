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
    // Boussinesq step (meshes with walls)
    unsigned char* wall_all = nullptr;  // [nd] 1 on every wall edge (no-slip velocity)
    double* tfoot = nullptr;  // [ne][N] semi-Lagrangian projection of the temperature
    double* gbt = nullptr;    // [ne][N] boundary-data vector of the temperature solve
    double* tdual = nullptr;  // [nd][Npsi] the temperature on the dual grid (buoyancy)
};

// Device bytes of a state's workspace.
inline uint64_t sld_state_bytes(const sld_state_s* st) {
    const uint64_t nd = uint64_t(st->disc->mesh->nd);
    const uint64_t nm = uint64_t(st->disc->mesh->ne) * st->disc->nphi;
    const uint64_t ndv = nd * 2 * st->disc->npsi;
    uint64_t b = 8 * (7 * nm + ndv);
    if (st->wall_all) b += nd + 8 * (2 * nm + nd * st->disc->npsi);
    return b;
}
