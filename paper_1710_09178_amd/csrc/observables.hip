// Polyakov loop: at every spatial site the ordered product of the time links
// around the periodic time direction, traced; block partials of the real and
// imaginary parts, summed in block order by the finaliser.
#include "observables.h"

namespace stag {

namespace {

__global__ __launch_bounds__(kBlock) void k_polyakov(Geom g, const double2* __restrict__ links,
                                                     double* __restrict__ part) {
    const int ns = g.nx * g.ny * g.nz;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < ns) {
        const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
        M3 P;
        for (int t = 0; t < g.nt; ++t) {
            const int par = (x + y + z + t) & 1;
            const double2* u = links + link_off(g, par, 3, 0) + cb_index(g, x, y, z, t);
            M3 U;
#pragma unroll
            for (int e = 0; e < 9; ++e) U.e[e] = u[(size_t)e * g.vh];
            P = (t == 0) ? U : m3_mul(P, U);
        }
        acc[0] = P.e[0].x + P.e[4].x + P.e[8].x;
        acc[1] = P.e[0].y + P.e[4].y + P.e[8].y;
    }
    block_partial<2>(acc, part);
}

}  // namespace

int launch_polyakov(const Geom& g, const double2* links, double* part, hipStream_t s) {
    const int grid = (g.nx * g.ny * g.nz + kBlock - 1) / kBlock;
    k_polyakov<<<grid, kBlock, 0, s>>>(g, links, part);
    return grid;
}

}  // namespace stag
