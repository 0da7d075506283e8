// Discrete velocity sets used by the HIP sweep (D2Q9, D3Q19), c_s^2 = 1/3.
//
// The speed of sound follows from the Maxwellian's covariance 1/(3 eps^2) I at
// eps = 1 (Sec. 3.3, Step 2, eq:homMaxwellianParametrized).  The sets and
// weights themselves are the textbook ones (part I of the paper leaves the
// lattice to its sequel).
//
// Ordering: rest first, then each velocity followed directly by its opposite,
// so opp(i) = i + 1 for odd i and i - 1 for even i > 0.  Axis directions
// precede diagonals.
#pragma once

namespace hlbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {
        1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

__host__ __device__ constexpr int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Index of the axis velocity +e_a (sign > 0) or -e_a (sign < 0) in lattice L.
template <class L>
__host__ __device__ constexpr int axis_velocity(int a, int sign)
{
    for (int i = 1; i < L::Q; ++i) {
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
        bool ok = c[a] == sign;
        for (int b = 0; b < 3; ++b)
            if (b != a && c[b] != 0) ok = false;
        if (ok) return i;
    }
    return -1;
}

}  // namespace hlbm
