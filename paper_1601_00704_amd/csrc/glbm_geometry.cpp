// Host-side geometry query of a class map: whether the open pores connect
// the two faces of the drive axis.  Near the site-percolation threshold of
// the lattice's neighbourhood the apparent permeability of a map is bimodal
// across seeds (an open-pore path or none), so a solve reports this flag
// beside k.
#include "glbm.h"

#include <cstdint>
#include <cstring>
#include <vector>

namespace glbm {
void set_error(const char* msg);  // glbm_api.cpp
}

extern "C" int glbm_pore_percolates(int32_t lattice, int32_t nx, int32_t ny, int32_t nz, const uint8_t* cls,
                                    int32_t axis, int32_t* percolates)
{
    glbm::set_error("");
    if (!cls || !percolates || nx < 1 || ny < 1 || nz < 1 || (lattice != GLBM_D2Q9 && lattice != GLBM_D3Q19) ||
        (lattice == GLBM_D2Q9 && nz != 1) || axis < 1 || axis > (lattice == GLBM_D2Q9 ? 2 : 3)) {
        glbm::set_error("glbm_pore_percolates: need a D2Q9 (nz = 1) or D3Q19 map of positive size and axis 1 .. 2 / 3");
        return GLBM_EINVAL;
    }
    const int64_t n = (int64_t)nx * ny * nz;
    const int a = axis - 1;
    const int dims[3] = {nx, ny, nz};
    // neighbour offsets: the lattice's non-rest velocities (D2Q9: 8, D3Q19: 18)
    std::vector<int> off;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int m = (dx != 0) + (dy != 0) + (dz != 0);
                if (m == 0) continue;
                if (lattice == GLBM_D2Q9 && dz != 0) continue;
                if (lattice == GLBM_D3Q19 && m == 3) continue;  // no corner velocities
                off.push_back(dx);
                off.push_back(dy);
                off.push_back(dz);
            }
    std::vector<uint8_t> seen((size_t)n, 0);
    std::vector<int64_t> queue;
    // seeds: open pores on the face at coordinate 0 of the drive axis
    for (int64_t i = 0; i < n; ++i) {
        const int c[3] = {int(i % nx), int((i / nx) % ny), int(i / ((int64_t)nx * ny))};
        if (c[a] == 0 && cls[i] == 0) {
            seen[i] = 1;
            queue.push_back(i);
        }
    }
    const int far = dims[a] - 1;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int64_t i = queue[h];
        const int c[3] = {int(i % nx), int((i / nx) % ny), int(i / ((int64_t)nx * ny))};
        if (c[a] == far) {
            *percolates = 1;
            return GLBM_OK;
        }
        for (size_t o = 0; o < off.size(); o += 3) {
            int q[3];
            bool inside = true;
            for (int d = 0; d < 3; ++d) {
                q[d] = c[d] + off[o + d];
                if (d == a) {
                    inside = inside && q[d] >= 0 && q[d] < dims[d];  // the drive axis does not wrap
                } else {
                    q[d] = (q[d] + dims[d]) % dims[d];  // the other axes are periodic
                }
            }
            if (!inside) continue;
            const int64_t j = ((int64_t)q[2] * ny + q[1]) * nx + q[0];
            if (cls[j] == 0 && !seen[j]) {
                seen[j] = 1;
                queue.push_back(j);
            }
        }
    }
    *percolates = 0;
    return GLBM_OK;
}
