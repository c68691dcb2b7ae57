// Exact reference-element matrices of the P_N AFE basis (Sec. 4.1, App. A)
// and the Gauss-Legendre time basis of the space-time predictor (Sec. 4.3).
//
// The Lagrange function of the lattice node with integer barycentric weights
// alpha (sum alpha_i = N) is built directly in product form,
//     phi_alpha = prod_i prod_{j < alpha_i} (N lambda_i - j) / (j + 1),
// which is one at its own node and zero at every other lattice node.  Each
// phi is expanded into monomials r^a s^b t^c with rational coefficients and
// integrated exactly with  int_T r^a s^b t^c = a! b! c! / (a+b+c+3)!  (and
// a! b! / (a+b+2)! on the reference triangle), so every matrix entry is an
// exact rational rounded once to double.
#include "refelem.hpp"

#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>

namespace afe {
namespace {

using i128 = __int128;

i128 gcd128(i128 a, i128 b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b != 0) {
        i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

struct Rat {
    i128 n = 0, d = 1;
    Rat() = default;
    Rat(long long v) : n(v), d(1) {}
    Rat(i128 a, i128 b) : n(a), d(b) { norm(); }
    void norm() {
        if (d < 0) { n = -n; d = -d; }
        i128 g = gcd128(n, d);
        if (g > 1) { n /= g; d /= g; }
        if (n == 0) d = 1;
    }
    Rat operator+(const Rat &o) const { return Rat(n * o.d + o.n * d, d * o.d); }
    Rat operator-(const Rat &o) const { return Rat(n * o.d - o.n * d, d * o.d); }
    Rat operator*(const Rat &o) const {
        i128 g1 = gcd128(n, o.d), g2 = gcd128(o.n, d);
        if (g1 == 0) g1 = 1;
        if (g2 == 0) g2 = 1;
        return Rat((n / g1) * (o.n / g2), (d / g2) * (o.d / g1));
    }
    bool zero() const { return n == 0; }
    double to_double() const {
        // exact for the magnitudes met here (|n|, d < 2^63): long double keeps 64 bits
        return static_cast<double>(static_cast<long double>(n) / static_cast<long double>(d));
    }
};

constexpr int kDeg = 9;  // total degree up to 2N = 8 (products of two basis functions at N = 4)
struct Poly {
    Rat c[kDeg][kDeg][kDeg];
    Poly() = default;
    static Poly constant(const Rat &v) {
        Poly p;
        p.c[0][0][0] = v;
        return p;
    }
    Poly operator*(const Poly &o) const {
        Poly r;
        for (int a = 0; a < kDeg; ++a)
            for (int b = 0; a + b < kDeg; ++b)
                for (int cc = 0; a + b + cc < kDeg; ++cc) {
                    if (c[a][b][cc].zero()) continue;
                    for (int x = 0; a + x < kDeg; ++x)
                        for (int y = 0; b + y < kDeg; ++y)
                            for (int z = 0; cc + z < kDeg && a + b + cc + x + y + z < kDeg; ++z) {
                                if (o.c[x][y][z].zero()) continue;
                                r.c[a + x][b + y][cc + z] = r.c[a + x][b + y][cc + z] + c[a][b][cc] * o.c[x][y][z];
                            }
                }
        return r;
    }
    Poly deriv(int dir) const {
        Poly r;
        for (int a = 0; a < kDeg; ++a)
            for (int b = 0; b < kDeg; ++b)
                for (int cc = 0; cc < kDeg; ++cc) {
                    if (c[a][b][cc].zero()) continue;
                    int e[3] = {a, b, cc};
                    if (e[dir] == 0) continue;
                    Rat f(static_cast<long long>(e[dir]));
                    e[dir] -= 1;
                    r.c[e[0]][e[1]][e[2]] = r.c[e[0]][e[1]][e[2]] + c[a][b][cc] * f;
                }
        return r;
    }
    double eval(double r, double s, double t) const {
        double v = 0.0;
        for (int a = 0; a < kDeg; ++a)
            for (int b = 0; b < kDeg; ++b)
                for (int cc = 0; cc < kDeg; ++cc)
                    if (!c[a][b][cc].zero()) v += c[a][b][cc].to_double() * std::pow(r, a) * std::pow(s, b) * std::pow(t, cc);
        return v;
    }
    Rat eval_exact(const Rat &r, const Rat &s, const Rat &t) const {
        Rat v;
        for (int a = 0; a < kDeg; ++a)
            for (int b = 0; b < kDeg; ++b)
                for (int cc = 0; cc < kDeg; ++cc) {
                    if (c[a][b][cc].zero()) continue;
                    Rat term = c[a][b][cc];
                    for (int i = 0; i < a; ++i) term = term * r;
                    for (int i = 0; i < b; ++i) term = term * s;
                    for (int i = 0; i < cc; ++i) term = term * t;
                    v = v + term;
                }
        return v;
    }
};

i128 fact(int k) {
    i128 f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

Rat tet_integral(const Poly &p) {
    Rat v;
    for (int a = 0; a < kDeg; ++a)
        for (int b = 0; b < kDeg; ++b)
            for (int c = 0; c < kDeg; ++c)
                if (!p.c[a][b][c].zero()) v = v + p.c[a][b][c] * Rat(fact(a) * fact(b) * fact(c), fact(a + b + c + 3));
    return v;
}

Rat tri_integral(const Poly &p) {  // over r, s >= 0, r + s <= 1 at t = 0
    Rat v;
    for (int a = 0; a < kDeg; ++a)
        for (int b = 0; b < kDeg; ++b)
            if (!p.c[a][b][0].zero()) v = v + p.c[a][b][0] * Rat(fact(a) * fact(b), fact(a + b + 2));
    return v;
}

// Lattice nodes N*(r, s, t) in the order of App. A.
std::vector<std::array<int, 3>> lattice(int N) {
    if (N == 1) return {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (N == 2)
        return {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 0, 0},
                {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}};
    if (N == 3)
        return {{0, 0, 0}, {3, 0, 0}, {0, 3, 0}, {0, 0, 3}, {1, 0, 0}, {2, 0, 0}, {2, 1, 0},
                {1, 2, 0}, {0, 2, 0}, {0, 1, 0}, {0, 0, 1}, {0, 0, 2}, {1, 0, 2}, {2, 0, 1},
                {0, 1, 2}, {0, 2, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
    if (N == 4) {
        // App. A.4 gives the quartic nodes only as the lattice; taken here:
        // the vertices in the order above, then the edge, face and interior
        // nodes, each group in lexicographic order of (r, s, t)
        std::vector<std::array<int, 3>> out = {{0, 0, 0}, {4, 0, 0}, {0, 4, 0}, {0, 0, 4}};
        for (int entity = 1; entity <= 3; ++entity)
            for (int i = 0; i <= 4; ++i)
                for (int j = 0; i + j <= 4; ++j)
                    for (int k = 0; i + j + k <= 4; ++k) {
                        const int l = 4 - i - j - k;
                        const int nz = (i > 0) + (j > 0) + (k > 0) + (l > 0);
                        if (nz - 1 == entity) out.push_back({i, j, k});
                    }
        return out;
    }
    throw std::invalid_argument("N must be 1, 2, 3 or 4");
}

// Legendre polynomial P_n and its derivative at x.
void legendre(int n, double x, double &p, double &dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void invert_small(const std::vector<double> &A, std::vector<double> &inv, int n) {
    std::vector<double> M(A);
    inv.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
        for (int k = 0; k < n; ++k) {
            std::swap(M[c * n + k], M[piv * n + k]);
            std::swap(inv[c * n + k], inv[piv * n + k]);
        }
        double d = M[c * n + c];
        for (int k = 0; k < n; ++k) { M[c * n + k] /= d; inv[c * n + k] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = M[r * n + c];
            for (int k = 0; k < n; ++k) { M[r * n + k] -= f * M[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
        }
    }
}

RefData build(int N) {
    RefData R;
    R.N = N;
    auto lat = lattice(N);
    R.np = static_cast<int>(lat.size());
    R.nt = N + 1;
    // barycentric polynomials
    Poly lam[4];
    lam[0] = Poly::constant(Rat(1));
    lam[0].c[1][0][0] = Rat(-1);
    lam[0].c[0][1][0] = Rat(-1);
    lam[0].c[0][0][1] = Rat(-1);
    lam[1].c[1][0][0] = Rat(1);
    lam[2].c[0][1][0] = Rat(1);
    lam[3].c[0][0][1] = Rat(1);
    std::vector<Poly> phi(R.np);
    for (int m = 0; m < R.np; ++m) {
        int a2 = lat[m][0], a3 = lat[m][1], a4 = lat[m][2];
        int a1 = N - a2 - a3 - a4;
        R.bary.push_back({a1, a2, a3, a4});
        R.xi.push_back({double(a2) / N, double(a3) / N, double(a4) / N});
        int al[4] = {a1, a2, a3, a4};
        Poly p = Poly::constant(Rat(1));
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < al[i]; ++j) {
                // (N lambda_i - j) / (j + 1)
                Poly f;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c)
                            if (!lam[i].c[a][b][c].zero()) f.c[a][b][c] = lam[i].c[a][b][c] * Rat(N, j + 1);
                f.c[0][0][0] = f.c[0][0][0] - Rat(j, j + 1);
                p = p * f;
            }
        phi[m] = p;
        if (lat[m][2] == 0) R.face_nodes.push_back(m);
    }
    R.nf = static_cast<int>(R.face_nodes.size());
    // nodal property check (exact)
    for (int m = 0; m < R.np; ++m)
        for (int l = 0; l < R.np; ++l) {
            Rat v = phi[l].eval_exact(Rat(lat[m][0], N), Rat(lat[m][1], N), Rat(lat[m][2], N));
            Rat want(static_cast<long long>(m == l ? 1 : 0));
            if ((v - want).n != 0) throw std::logic_error("nodal property violated");
        }
    std::vector<Poly> dphi[3];
    for (int d = 0; d < 3; ++d)
        for (int l = 0; l < R.np; ++l) dphi[d].push_back(phi[l].deriv(d));
    const int np = R.np;
    R.M.assign(np * np, 0.0);
    R.K.assign(3 * np * np, 0.0);
    R.D.assign(3 * np * np, 0.0);
    for (int m = 0; m < np; ++m)
        for (int l = 0; l < np; ++l) {
            R.M[m * np + l] = tet_integral(phi[m] * phi[l]).to_double();
            for (int d = 0; d < 3; ++d) {
                R.K[(d * np + m) * np + l] = tet_integral(phi[m] * dphi[d][l]).to_double();
                R.D[(d * np + m) * np + l] =
                    dphi[d][l].eval_exact(Rat(lat[m][0], N), Rat(lat[m][1], N), Rat(lat[m][2], N)).to_double();
            }
        }
    const int nf = R.nf;
    R.Z.assign(nf * nf, 0.0);
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) R.Z[i * nf + j] = tri_integral(phi[R.face_nodes[i]] * phi[R.face_nodes[j]]).to_double();
    // Gauss-Legendre nodes on [-1, 1] by Newton's method, mapped to [0, 1]
    const int nt = R.nt;
    R.tau.assign(nt, 0.0);
    R.w.assign(nt, 0.0);
    for (int i = 0; i < nt; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (nt + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(nt, x, p, dp);
            double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        double p, dp;
        legendre(nt, x, p, dp);
        // ascending order on [0, 1]
        R.tau[nt - 1 - i] = 0.5 * (x + 1.0);
        R.w[nt - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2 / ((1-x^2) P'^2)) / 2
    }
    // Lagrange time basis psi_a through tau; K_tau[a][b] = psi_a(1) psi_b(1) - int psi_a' psi_b
    auto psi = [&](int a, double s) {
        double v = 1.0;
        for (int b = 0; b < nt; ++b)
            if (b != a) v *= (s - R.tau[b]) / (R.tau[a] - R.tau[b]);
        return v;
    };
    auto dpsi = [&](int a, double s) {
        double tot = 0.0;
        for (int c = 0; c < nt; ++c) {
            if (c == a) continue;
            double v = 1.0 / (R.tau[a] - R.tau[c]);
            for (int b = 0; b < nt; ++b)
                if (b != a && b != c) v *= (s - R.tau[b]) / (R.tau[a] - R.tau[b]);
            tot += v;
        }
        return tot;
    };
    R.Ktau.assign(nt * nt, 0.0);
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            // int_0^1 psi_a' psi_b: degree 2N-1, exact with the N+1 point rule
            double integ = 0.0;
            for (int c = 0; c < nt; ++c) integ += R.w[c] * dpsi(a, R.tau[c]) * psi(b, R.tau[c]);
            R.Ktau[a * nt + b] = psi(a, 1.0) * psi(b, 1.0) - integ;
        }
    invert_small(R.Ktau, R.Ktau_inv, nt);
    // conical product rule for error norms: n-point Gauss-Legendre on [0, 1]
    // in each collapsed coordinate, n = N + 3
    const int ng = N + 3;
    std::vector<double> gx(ng), gw(ng);
    for (int i = 0; i < ng; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (ng + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(ng, x, p, dp);
            const double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        double p, dp;
        legendre(ng, x, p, dp);
        gx[i] = 0.5 * (x + 1.0);
        gw[i] = 1.0 / ((1.0 - x * x) * dp * dp);
    }
    R.nq = ng * ng * ng;
    for (int ia = 0; ia < ng; ++ia)
        for (int ib = 0; ib < ng; ++ib)
            for (int ic = 0; ic < ng; ++ic) {
                const double a = gx[ia], b = gx[ib], c = gx[ic];
                const double xi[3] = {a * (1.0 - b) * (1.0 - c), b * (1.0 - c), c};
                R.qxi.insert(R.qxi.end(), xi, xi + 3);
                R.qw.push_back(gw[ia] * gw[ib] * gw[ic] * (1.0 - b) * (1.0 - c) * (1.0 - c));
                for (int m = 0; m < R.np; ++m) R.qphi.push_back(phi[m].eval(xi[0], xi[1], xi[2]));
            }
    return R;
}

}  // namespace

const RefData &ref_data(int N) {
    static std::mutex mu;
    static std::map<int, RefData> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(N);
    if (it == cache.end()) it = cache.emplace(N, build(N)).first;
    return it->second;
}

}  // namespace afe
