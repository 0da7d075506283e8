// Host check of the row classification of boxes with walls or open faces that
// the sweep and reverse-step kernels use: against a brute-force reading of the
// pull rule (the source of direction c at x is x - c, wrapped on a periodic
// axis; a pull crosses a face when that source lies beyond an open face or in
// a wall's solid layer), over many box shapes and face kinds:
//   * plain_row(y, z) holds exactly when no cell of the row lies in a y or z
//     wall layer and no pull of a cell of the row crosses a y or z face;
//   * on a plain row, a fluid cell's pull in direction c crosses an x face
//     exactly when c_x = +1 and x = x_end_lo, or c_x = -1 and x = x_end_hi;
//   * row_of is a bijection of the rows that lists every row that is not
//     plain before every plain row.
#include <cstdio>
#include <vector>

#include "../../paper_2310_14746_amd/csrc/hlbm_internal.hpp"

using namespace hlbm;

struct Axis {
    int n, lo, hi;  // size, face kinds (0 periodic, 1 wall, 2 inlet, 3 outlet)
    bool wall_layer(int s) const { return (lo == 1 && s == 0) || (hi == 1 && s == n - 1); }
    // whether the pull from coordinate X with velocity component c crosses a face
    bool crosses(int X, int c) const
    {
        int s = X - c;
        if (lo == 0) s = (s + n) % n;
        if (s < 0 || s >= n) return true;
        return wall_layer(s);
    }
};

static int check(const Axis& ax, const Axis& ay, const Axis& az)
{
    int bad = 0;
    for (int z = 0; z < az.n; ++z)
        for (int y = 0; y < ay.n; ++y) {
            bool expect = !(ay.wall_layer(y) || az.wall_layer(z));
            for (int cy = -1; cy <= 1; ++cy)
                for (int cz = -1; cz <= 1; ++cz)
                    if (ay.crosses(y, cy) || az.crosses(z, cz)) expect = false;
            const bool got = plain_row(y, z, ay.n, az.n, ay.lo, ay.hi, az.lo, az.hi);
            if (got != expect) {
                if (bad++ < 5)
                    printf("row (%d,%d) of %dx%dx%d kinds %d%d/%d%d: plain_row %d, expected %d\n", y, z, ax.n, ay.n,
                           az.n, ay.lo, ay.hi, az.lo, az.hi, got, expect);
                continue;
            }
            if (!got) continue;
            const int xl = x_end_lo(ax.lo), xh = x_end_hi(ax.hi, ax.n);
            for (int x = 0; x < ax.n; ++x) {
                if (ax.wall_layer(x)) continue;  // solid: its pulls are discarded
                for (int cx = -1; cx <= 1; ++cx) {
                    const bool cross = ax.crosses(x, cx);
                    const bool fixed = (cx == 1 && x == xl) || (cx == -1 && x == xh);
                    if (cross != fixed && bad++ < 5)
                        printf("x=%d c_x=%d of nx=%d kinds %d/%d: crosses %d, x-end fix %d\n", x, cx, ax.n, ax.lo,
                               ax.hi, cross, fixed);
                }
            }
        }
    // row order: a bijection, rows that are not plain first
    std::vector<int> seen(ay.n * az.n, 0);
    bool plain_seen = false;
    for (int r = 0; r < ay.n * az.n; ++r) {
        int y = -1, z = -1;
        row_of(r, ay.n, az.n, ay.lo, ay.hi, az.lo, az.hi, y, z);
        if (y < 0 || y >= ay.n || z < 0 || z >= az.n) {
            if (bad++ < 5) printf("row_of(%d) = (%d,%d) outside %dx%d\n", r, y, z, ay.n, az.n);
            continue;
        }
        seen[y + ay.n * z]++;
        const bool pl = plain_row(y, z, ay.n, az.n, ay.lo, ay.hi, az.lo, az.hi);
        if (!pl && plain_seen && bad++ < 5) printf("row_of(%d): a row that is not plain after a plain one\n", r);
        plain_seen |= pl;
    }
    for (int k = 0; k < ay.n * az.n; ++k)
        if (seen[k] != 1 && bad++ < 5) printf("row %d of %dx%d listed %d times\n", k, ay.n, az.n, seen[k]);
    return bad;
}

int main()
{
    // face-kind pairs per axis (lo, hi); periodic faces come in pairs
    const int pairs[][2] = {{0, 0}, {1, 1}, {2, 3}, {3, 2}, {1, 2}, {3, 1}, {2, 2}};
    int cases = 0, failed = 0;
    for (const auto& kx : pairs)
        for (const auto& ky : pairs)
            for (const auto& kz : pairs)
                for (int nx : {1, 2, 3, 4, 5, 9, 16})
                    for (int ny : {1, 2, 3, 4, 5, 7})
                        for (int nz : {1, 2, 3, 5}) {
                            ++cases;
                            if (check(Axis{nx, kx[0], kx[1]}, Axis{ny, ky[0], ky[1]}, Axis{nz, kz[0], kz[1]})) ++failed;
                        }
    printf("%d cases, %d failed\n", cases, failed);
    return failed != 0;
}
