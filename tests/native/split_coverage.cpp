// Host check of the interior/shell decomposition used by the adjoint sweep:
// for many box shapes and face kinds, the interior sub-box plus the shell
// cells enumerated by shell_cell() -- and the one-launch block mapping of
// adjoint_split_kernel -- cover every cell exactly once, and every shell cell
// lies within two layers of a wall face or one layer of an open face.
#include <cstdio>
#include <vector>

#include "../../paper_2310_14746_amd/csrc/hlbm_internal.hpp"

using namespace hlbm;

static int check(int nx, int ny, int nz, const int lo[3], const int hi[3], int bx)
{
    Params p = {};
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.N = (uint32_t)(nx * ny * nz);
    for (int a = 0; a < 3; ++a) {
        p.bc_lo[a] = lo[a];
        p.bc_hi[a] = hi[a];
    }
    const Split s = split_of(p, bx);
    if (!s.interior()) return 0;  // the general kernel covers every cell
    std::vector<int> hit(p.N, 0);
    const int n[3] = {nx, ny, nz};
    for (uint32_t b = 0; b < s.blocks_shell + s.blocks_in; ++b)
        for (uint32_t t = 0; t < (uint32_t)bx; ++t) {
            uint32_t x, y, z;
            bool shell = b < s.blocks_shell;
            if (shell) {
                const uint32_t k = b * bx + t;
                if (k >= s.n_shell) continue;
                shell_cell(s, nx, ny, k, x, y, z);
            } else {
                const uint32_t bi = b - s.blocks_shell, row = bi / s.gx, bxi = bi - row * s.gx;
                const uint32_t iy = s.hi[1] - s.lo[1], zz = row / iy, yy = row - zz * iy;
                x = s.lo[0] + bxi * bx + t;
                if (x >= s.hi[0]) continue;
                y = s.lo[1] + yy;
                z = s.lo[2] + zz;
            }
            if (x >= (uint32_t)nx || y >= (uint32_t)ny || z >= (uint32_t)nz) {
                printf("out of range: %dx%dx%d bx %d\n", nx, ny, nz, bx);
                return 1;
            }
            const uint32_t c[3] = {x, y, z};
            bool near = false;
            for (int a = 0; a < 3; ++a) {
                if (lo[a] == 0) continue;
                const uint32_t dl = lo[a] == 1 ? 2u : 1u, dh = hi[a] == 1 ? 2u : 1u;
                if (c[a] < dl || c[a] + dh >= (uint32_t)n[a]) near = true;
            }
            if (shell != near) {
                printf("cell (%u,%u,%u) of %dx%dx%d: shell %d, near a face %d\n", x, y, z, nx, ny, nz, shell, near);
                return 1;
            }
            hit[x + nx * (y + ny * z)]++;
        }
    for (uint32_t k = 0; k < p.N; ++k)
        if (hit[k] != 1) {
            printf("cell %u of %dx%dx%d covered %d times\n", k, nx, ny, nz, hit[k]);
            return 1;
        }
    return 0;
}

int main()
{
    // face kinds per axis (lo, hi): 0 periodic, 1 wall, 2 inlet, 3 outlet
    const int kinds[][6] = {{0, 0, 0, 0, 0, 0}, {0, 1, 1, 0, 1, 1}, {2, 1, 1, 3, 1, 1}, {0, 1, 0, 0, 1, 0},
                            {1, 0, 0, 1, 0, 0}, {0, 0, 1, 0, 0, 1}, {2, 0, 0, 3, 0, 0}, {2, 1, 0, 3, 1, 0},
                            {1, 1, 1, 1, 1, 1}, {1, 2, 1, 1, 3, 1}, {3, 0, 2, 2, 0, 3}};
    int cases = 0, bad = 0;
    for (const auto& k : kinds)
        for (int nx : {3, 4, 5, 6, 9, 16, 70})
            for (int ny : {3, 4, 5, 7, 12})
                for (int nz : {1, 3, 5, 8})
                    for (int bx : {64, 128}) {
                        const int lo[3] = {k[0], k[1], k[2]}, hi[3] = {k[3], k[4], k[5]};
                        if (nz == 1 && lo[2] != 0) continue;
                        ++cases;
                        bad += check(nx, ny, nz, lo, hi, bx);
                    }
    printf("%d cases, %d failed\n", cases, bad);
    return bad != 0;
}
