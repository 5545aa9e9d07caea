// FP64 host-side set-up arithmetic of libpic.so: collision-frequency tables,
// the charge-form finite-volume couplings of the R-Z field operator, node
// kinds, node volumes and the dense inverse for the coarsest multigrid level.
// Built with -ffp-contract=off so the values do not depend on FMA fusion.
#include <cmath>
#include <vector>

#include "common.h"

namespace pic {

namespace {
constexpr double kEps0 = 8.8541878128e-12;   // CODATA 2018
constexpr double kQe = 1.602176634e-19;
constexpr double kKb = 1.380649e-23;
constexpr double kPi = 3.14159265358979323846;
}  // namespace

// Null-collision tables (Section 3's processes (1a)-(1c) against a static
// argon background of density n_g = p / (k_B T), (1d) against the static
// metastable density n_meta):
//   nu_c(E_k) = n_c sigma_c(E_k) v(E_k),  v = sqrt(2 e E / m_e),
//   nu_max   = max_k sum_c nu_c(E_k)  (bounds the piecewise-linear interpolant),
//   t_null   = floor((1 - exp(-nu_max dt)) 2^32)  (candidate iff u0 < t_null).
double host_nu_tables(const pic_config &c, double *nu, unsigned long long *t_null)
{
    const double ng = c.p_gas / (kKb * c.t_gas);
    double numax = 0.0;
    for (int k = 0; k < c.n_table; ++k) {
        const double e = k * c.de_table;
        const double v = std::sqrt(2.0 * kQe * e / c.m[0]);
        double sum = 0.0;
        for (int p = 0; p < 4; ++p) {
            const double target = (p < 3) ? ng : c.n_meta;
            nu[p * c.n_table + k] = target * c.sigma[p * c.n_table + k] * v;
            sum += nu[p * c.n_table + k];
        }
        if (sum > numax) numax = sum;
    }
    const double pnull = 1.0 - std::exp(-numax * c.dt);
    *t_null = (unsigned long long)std::floor(pnull * 4294967296.0);
    return numax;
}

// Emission threshold: an absorbed particle of species s (yield gamma_e for
// electrons, gamma_i for ions) emits one electron iff its draw
// u0 < floor(min(1, gamma w_s / w_e) 2^32).
unsigned long long host_see_threshold(const pic_config &c, int species)
{
    double p = (species == 0 ? c.gamma_e : c.gamma_i) * c.w[species] / c.w[0];
    if (p > 1.0) p = 1.0;
    if (p < 0.0) p = 0.0;
    return (unsigned long long)std::floor(p * 4294967296.0);
}

int host_node_kind(int nr, int nz, double lr, double cathode_rmax, int i, int j)
{
    const double r = i * (lr / nr);
    if (j == nz || i == nr) return 2;
    if (j == 0 && r < cathode_rmax) return 1;
    return 0;
}

// Couplings scale * A_f / h_f of the control-volume faces (the reading of
// Section 3's "Gauss' law is obeyed along this axis"): node (i, j) owns
// [r_{i-1/2}, r_{i+1/2}] x [z_{j-1/2}, z_{j+1/2}] clipped to the domain.
//   east  face (i+1/2): area 2 pi r_{i+1/2} dz_j, dz_j halved on z walls;
//   north face (j+1/2): area pi (r_hi^2 - r_lo^2) of the node's annulus.
void host_couplings(int nr, int nz, double lr, double lz, double scale, double *ce, double *cn)
{
    const double dr = lr / nr, dz = lz / nz;
    for (int j = 0; j <= nz; ++j) {
        for (int i = 0; i <= nr; ++i) {
            const long n = (long)j * (nr + 1) + i;
            if (i < nr) {
                const double hz = (j == 0 || j == nz) ? 0.5 * dz : dz;
                ce[n] = scale * (2.0 * kPi * ((i + 0.5) * dr) * hz) / dr;
            } else {
                ce[n] = 0.0;
            }
            if (j < nz) {
                const double lo = (i == 0) ? 0.0 : (i - 0.5) * dr;
                const double hi = (i == nr) ? lr : (i + 0.5) * dr;
                cn[n] = scale * (kPi * (hi * hi - lo * lo)) / dz;
            } else {
                cn[n] = 0.0;
            }
        }
    }
}

// Volume integral of the node's tent weight (linear in r and z):
//   axis pi dr^2/3, interior 2 pi r_i dr, outer wall pi dr R - pi dr^2/3,
// times dz (dz/2 on the z walls).  Q / (q V) is then the number density
// that a uniform load reproduces at every node.
void host_node_volumes(int nr, int nz, double lr, double lz, double *v)
{
    const double dr = lr / nr, dz = lz / nz;
    for (int j = 0; j <= nz; ++j) {
        const double hz = (j == 0 || j == nz) ? 0.5 * dz : dz;
        for (int i = 0; i <= nr; ++i) {
            double a;
            if (i == 0) a = kPi * dr * dr / 3.0;
            else if (i == nr) a = kPi * dr * lr - kPi * dr * dr / 3.0;
            else a = 2.0 * kPi * (i * dr) * dr;
            v[(long)j * (nr + 1) + i] = a * hz;
        }
    }
}

// Gauss-Jordan inverse with partial pivoting, in place (row-major n x n).
int host_dense_inverse(int n, double *a)
{
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + col]) > std::fabs(a[(size_t)piv * n + col])) piv = r;
        if (a[(size_t)piv * n + col] == 0.0) return -1;
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
                std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
            }
        const double d = 1.0 / a[(size_t)col * n + col];
        for (int k = 0; k < n; ++k) {
            a[(size_t)col * n + k] *= d;
            inv[(size_t)col * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = a[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)col * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
            }
        }
    }
    for (size_t k = 0; k < (size_t)n * n; ++k) a[k] = inv[k];
    return 0;
}

double eps0() { return kEps0; }

}  // namespace pic
