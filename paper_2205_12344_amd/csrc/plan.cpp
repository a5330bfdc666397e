// Host-side set-up of libelwh: argument checks, padded layout, stencil
// constants, the metric terms of mapped grids and the time-step plan.
//
// Time-step rule (the paper fixes only a CFL number for explicit FD runs,
// Sec. 5.1, and a whole number of steps per period for the implicit scheme,
// Sec. 4.4): G = max over unknown rows of sum_j |(rho^-1 Ltilde)_ij|
// (Gershgorin), dt* = cfl * 2 / sqrt(G), N_T = max(3, ceil(T / dt*)),
// dt = T / N_T, and the correction factor c = (sin(w dt/2) / (w dt/2))^2 of
// the corrected scheme (Sec. 4.3).
//
// The rows of Ltilde are those of minus the Hessian of the discrete strain
// energy (trapezoid rule; edge terms 1/2 w_e k_e (D+ u)^2, node terms
// w_p [lam (Dh_a u_a)(Dh_b u_b) + mu (Dh_b u_a)(Dh_a u_b)]), divided by the
// node weight.  Rows two or more cells away from every face use the closed
// form of the conservative stencil; rows near a face enumerate the energy
// terms that touch them.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "elwh_internal.h"

namespace elwh {

namespace {

struct Geo {
    int d;
    int n[3];
    double h[3];
    int bc[6];
    int64_t sx, sy, sz;  // caller-layout strides
    const double *rho, *lam, *mu;

    bool unknown(const int* p) const {
        for (int a = 0; a < d; ++a) {
            if (p[a] == 0 && bc[2 * a] == ELWH_BC_DIRICHLET) return false;
            if (p[a] == n[a] && bc[2 * a + 1] == ELWH_BC_DIRICHLET) return false;
        }
        return true;
    }
    bool inside(const int* p) const {
        for (int a = 0; a < d; ++a)
            if (p[a] < 0 || p[a] > n[a]) return false;
        return true;
    }
    int64_t idx(const int* p) const { return p[0] * sx + p[1] * sy + (d == 3 ? p[2] * sz : 0); }
    double node_w(const int* p) const {
        double w = 1.0;
        for (int a = 0; a < d; ++a) {
            if (p[a] == 0 && bc[2 * a] == ELWH_BC_TRACTION_FREE) w *= 0.5;
            if (p[a] == n[a] && bc[2 * a + 1] == ELWH_BC_TRACTION_FREE) w *= 0.5;
        }
        return w;
    }
    // weight of the edge from p along axis a: 1/2 per free face of another axis
    double edge_w(const int* p, int a) const {
        double w = 1.0;
        for (int b = 0; b < d; ++b) {
            if (b == a) continue;
            if (p[b] == 0 && bc[2 * b] == ELWH_BC_TRACTION_FREE) w *= 0.5;
            if (p[b] == n[b] && bc[2 * b + 1] == ELWH_BC_TRACTION_FREE) w *= 0.5;
        }
        return w;
    }
    // node difference Dh_a at q: up to two (node, coefficient) pairs
    int dhat(const int* q, int a, int nodes[2][3], double coef[2]) const {
        int k = 0;
        auto put = [&](int off, double cf) {
            for (int b = 0; b < 3; ++b) nodes[k][b] = q[b];
            nodes[k][a] += off;
            coef[k] = cf;
            ++k;
        };
        if (q[a] == 0) {
            if (bc[2 * a] == ELWH_BC_TRACTION_FREE) { put(1, 1.0 / h[a]); put(0, -1.0 / h[a]); }
        } else if (q[a] == n[a]) {
            if (bc[2 * a + 1] == ELWH_BC_TRACTION_FREE) { put(0, 1.0 / h[a]); put(-1, -1.0 / h[a]); }
        } else {
            put(1, 0.5 / h[a]);
            put(-1, -0.5 / h[a]);
        }
        return k;
    }
};

// Gershgorin row sum of rho^-1 Ltilde for dof (p, c), from the energy terms.
double row_sum_generic(const Geo& g, const int* p, int c) {
    // K row entries keyed by neighbour offset in {-1,0,1}^3 and component
    double K[27][3];
    std::memset(K, 0, sizeof(K));
    auto slot = [&](const int* t) {
        return (t[0] - p[0] + 1) + 3 * (t[1] - p[1] + 1) + 9 * ((g.d == 3 ? t[2] - p[2] : 0) + 1);
    };
    const int d = g.d;
    // compact edge terms touching p, component c
    for (int a = 0; a < d; ++a) {
        for (int side = 0; side < 2; ++side) {
            int lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
            if (side == 0) {
                if (p[a] == 0) continue;
                lo[a] -= 1;
            } else {
                if (p[a] == g.n[a]) continue;
                hi[a] += 1;
            }
            const int64_t il = g.idx(lo), ih = g.idx(hi);
            double k;
            if (c == a)
                k = 0.5 * ((g.lam[il] + 2 * g.mu[il]) + (g.lam[ih] + 2 * g.mu[ih]));
            else
                k = 0.5 * (g.mu[il] + g.mu[ih]);
            const double e = g.edge_w(lo, a) * k / (g.h[a] * g.h[a]);
            const int* other = side == 0 ? lo : hi;
            K[slot(p)][c] += e;
            K[slot(other)][c] -= e;
        }
    }
    // node cross terms at q = p and q = p +- e_x (the only nodes whose node
    // differences involve p)
    std::vector<std::array<int, 3>> qs;
    qs.push_back({p[0], p[1], p[2]});
    for (int a = 0; a < d; ++a)
        for (int s = -1; s <= 1; s += 2) {
            std::array<int, 3> q = {p[0], p[1], p[2]};
            q[a] += s;
            qs.push_back(q);
        }
    for (auto& qa : qs) {
        const int* q = qa.data();
        if (!g.inside(q) || !g.unknown(q)) continue;
        const int64_t iq = g.idx(q);
        const double wq = g.node_w(q);
        for (int a = 0; a < d; ++a)
            for (int b = a + 1; b < d; ++b) {
                int na[2][3], nb[2][3];
                double ca_[2], cb_[2];
                const int ka = g.dhat(q, a, na, ca_);
                const int kb = g.dhat(q, b, nb, cb_);
                // term coef * (D1 u_alpha)(D2 u_beta)
                struct Term { double coef; int alpha, beta; bool d1_is_a; };
                const Term terms[2] = {{wq * g.lam[iq], a, b, true},    // lam (Dh_a u_a)(Dh_b u_b)
                                       {wq * g.mu[iq], a, b, false}};   // mu (Dh_b u_a)(Dh_a u_b)
                for (const Term& t : terms) {
                    int (*n1)[3] = t.d1_is_a ? na : nb;
                    int (*n2)[3] = t.d1_is_a ? nb : na;
                    const double* c1 = t.d1_is_a ? ca_ : cb_;
                    const double* c2 = t.d1_is_a ? cb_ : ca_;
                    const int k1 = t.d1_is_a ? ka : kb, k2 = t.d1_is_a ? kb : ka;
                    if (c == t.alpha)
                        for (int s = 0; s < k1; ++s)
                            if (n1[s][0] == p[0] && n1[s][1] == p[1] && n1[s][2] == p[2])
                                for (int r = 0; r < k2; ++r) K[slot(n2[r])][t.beta] += t.coef * c1[s] * c2[r];
                    if (c == t.beta)
                        for (int s = 0; s < k2; ++s)
                            if (n2[s][0] == p[0] && n2[s][1] == p[1] && n2[s][2] == p[2])
                                for (int r = 0; r < k1; ++r) K[slot(n1[r])][t.alpha] += t.coef * c2[s] * c1[r];
                }
            }
    }
    // Ltilde = -K / w_p over unknown targets
    double sum = 0.0;
    const int zr = d == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int t[3] = {p[0] + dx, p[1] + dy, p[2] + dz};
                if (!g.inside(t) || !g.unknown(t)) continue;
                for (int cc = 0; cc < d; ++cc) sum += std::fabs(K[slot(t)][cc]);
            }
    return sum / g.node_w(p) / g.rho[g.idx(p)];
}

// Closed-form row sums (all components) for a node two or more cells from
// every face: every stencil entry is a sum of positive coefficients.
double row_sum_interior(const Geo& g, const int* p) {
    const int64_t C = g.idx(p);
    auto at = [&](const double* a, int dx, int dy, int dz) {
        return a[C + dx * g.sx + dy * g.sy + dz * g.sz];
    };
    const double hx = g.h[0], hy = g.h[1];
    const double ixx = 1 / (hx * hx), iyy = 1 / (hy * hy), ixy = 1 / (2 * hx * hy);
    auto A = [&](int dx, int dy, int dz) { return at(g.lam, dx, dy, dz) + 2 * at(g.mu, dx, dy, dz); };
    auto M = [&](int dx, int dy, int dz) { return at(g.mu, dx, dy, dz); };
    auto Lm = [&](int dx, int dy, int dz) { return at(g.lam, dx, dy, dz); };
    double best;
    if (g.d == 2) {
        const double ru = (A(1, 0, 0) + 2 * A(0, 0, 0) + A(-1, 0, 0)) * ixx +
                          (M(0, 1, 0) + 2 * M(0, 0, 0) + M(0, -1, 0)) * iyy +
                          (Lm(1, 0, 0) + Lm(-1, 0, 0) + M(0, 1, 0) + M(0, -1, 0)) * ixy;
        const double rv = (M(1, 0, 0) + 2 * M(0, 0, 0) + M(-1, 0, 0)) * ixx +
                          (A(0, 1, 0) + 2 * A(0, 0, 0) + A(0, -1, 0)) * iyy +
                          (M(1, 0, 0) + M(-1, 0, 0) + Lm(0, 1, 0) + Lm(0, -1, 0)) * ixy;
        best = std::max(ru, rv);
    } else {
        const double hz = g.h[2];
        const double izz = 1 / (hz * hz), ixz = 1 / (2 * hx * hz), iyz = 1 / (2 * hy * hz);
        const double ru = (A(1, 0, 0) + 2 * A(0, 0, 0) + A(-1, 0, 0)) * ixx +
                          (M(0, 1, 0) + 2 * M(0, 0, 0) + M(0, -1, 0)) * iyy +
                          (M(0, 0, 1) + 2 * M(0, 0, 0) + M(0, 0, -1)) * izz +
                          (Lm(1, 0, 0) + Lm(-1, 0, 0) + M(0, 1, 0) + M(0, -1, 0)) * ixy +
                          (Lm(1, 0, 0) + Lm(-1, 0, 0) + M(0, 0, 1) + M(0, 0, -1)) * ixz;
        const double rv = (M(1, 0, 0) + 2 * M(0, 0, 0) + M(-1, 0, 0)) * ixx +
                          (A(0, 1, 0) + 2 * A(0, 0, 0) + A(0, -1, 0)) * iyy +
                          (M(0, 0, 1) + 2 * M(0, 0, 0) + M(0, 0, -1)) * izz +
                          (M(1, 0, 0) + M(-1, 0, 0) + Lm(0, 1, 0) + Lm(0, -1, 0)) * ixy +
                          (Lm(0, 1, 0) + Lm(0, -1, 0) + M(0, 0, 1) + M(0, 0, -1)) * iyz;
        const double rw = (M(1, 0, 0) + 2 * M(0, 0, 0) + M(-1, 0, 0)) * ixx +
                          (M(0, 1, 0) + 2 * M(0, 0, 0) + M(0, -1, 0)) * iyy +
                          (A(0, 0, 1) + 2 * A(0, 0, 0) + A(0, 0, -1)) * izz +
                          (M(1, 0, 0) + M(-1, 0, 0) + Lm(0, 0, 1) + Lm(0, 0, -1)) * ixz +
                          (M(0, 1, 0) + M(0, -1, 0) + Lm(0, 0, 1) + Lm(0, 0, -1)) * iyz;
        best = std::max(ru, std::max(rv, rw));
    }
    return best / g.rho[C];
}

double gershgorin(const Geo& g) {
    const int nzn = g.d == 3 ? g.n[2] + 1 : 1;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, (unsigned)nzn * (g.d == 3 ? 1 : 1));
    if (g.d == 2) nth = std::min<unsigned>(nth, (unsigned)(g.n[1] + 1));
    std::vector<double> part(nth, 0.0);
    auto work = [&](unsigned t) {
        double best = 0.0;
        const int outer = g.d == 3 ? nzn : g.n[1] + 1;
        for (int o = (int)t; o < outer; o += (int)nth) {
            int p[3] = {0, 0, 0};
            const int ylo = g.d == 3 ? 0 : o, yhi = g.d == 3 ? g.n[1] : o;
            if (g.d == 3) p[2] = o;
            for (int y = ylo; y <= yhi; ++y) {
                p[1] = y;
                for (int x = 0; x <= g.n[0]; ++x) {
                    p[0] = x;
                    if (!g.unknown(p)) continue;
                    bool near = false;
                    for (int a = 0; a < g.d; ++a)
                        if (p[a] < 2 || p[a] > g.n[a] - 2) near = true;
                    double r;
                    if (near) {
                        r = 0.0;
                        for (int c = 0; c < g.d; ++c) r = std::max(r, row_sum_generic(g, p, c));
                    } else {
                        r = row_sum_interior(g, p);
                    }
                    best = std::max(best, r);
                }
            }
        }
        part[t] = best;
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nth; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& x : th) x.join();
    return *std::max_element(part.begin(), part.end());
}

// ---- mapped 2-D grids ---------------------------------------------------------

// Second-order derivative of node values along one index direction (stride
// st, n+1 nodes, spacing h): central inside, one-sided over three nodes at
// both ends.
double diff1(const double* f, int64_t o, int64_t st, int k, int n, double h) {
    if (k == 0) return (-3.0 * f[o] + 4.0 * f[o + st] - f[o + 2 * st]) / (2.0 * h);
    if (k == n) return (3.0 * f[o] - 4.0 * f[o - st] + f[o - 2 * st]) / (2.0 * h);
    return (f[o + st] - f[o - st]) / (2.0 * h);
}

// The 2x2 blocks K^qq, K^qr, K^rr at one node (row-major [i][k]).
void mapped_blocks(const MappedMetric& m, const double* lam, const double* mu, int64_t o, double qq[4],
                   double qr[4], double rr[4]) {
    const double l = lam[o] / m.J[o], u = mu[o] / m.J[o], lu = l + u;
    const double A0 = m.g[0][o], A1 = m.g[1][o], B0 = m.g[2][o], B1 = m.g[3][o];
    const double AA = A0 * A0 + A1 * A1, BB = B0 * B0 + B1 * B1, AB = A0 * B0 + A1 * B1;
    qq[0] = lu * A0 * A0 + u * AA; qq[1] = lu * A0 * A1; qq[2] = qq[1]; qq[3] = lu * A1 * A1 + u * AA;
    rr[0] = lu * B0 * B0 + u * BB; rr[1] = lu * B0 * B1; rr[2] = rr[1]; rr[3] = lu * B1 * B1 + u * BB;
    qr[0] = lu * A0 * B0 + u * AB; qr[1] = l * A0 * B1 + u * B0 * A1;
    qr[2] = l * A1 * B0 + u * B1 * A0; qr[3] = lu * A1 * B1 + u * AB;
}

// Gershgorin row sums of (w_p rho J)^-1 L_h on a mapped grid (q sides
// Dirichlet, r sides Dirichlet or traction-free): the stencil entries of
// each unknown row, summed per (neighbour, component) before taking absolute
// values.  A traction-free row (weight 1/2) is the Hessian row of the
// energy with the one-sided r difference in its cross terms, times 2.
double gershgorin_mapped(int nq, int nr, const MappedMetric& m, const double* rho, const double* lam,
                         const double* mu, bool free_lo, bool free_hi) {
    const double hq = 1.0 / nq, hr = 1.0 / nr;
    const double iqq = 1.0 / (hq * hq), irr = 1.0 / (hr * hr), iqr = 1.0 / (4.0 * hq * hr);
    const int64_t sy = nq + 1;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int jlo = free_lo ? 0 : 1, jhi = free_hi ? nr : nr - 1;
    nth = std::min<unsigned>(nth, (unsigned)std::max(1, jhi - jlo + 1));
    std::vector<double> part(nth, 0.0);
    auto work = [&](unsigned t) {
        double best = 0.0;
        for (int j = jlo + (int)t; j <= jhi; j += (int)nth)
            for (int i = 1; i <= nq - 1; ++i) {
                const int64_t p = j * sy + i;
                double E[3][3][2][2];   // [dj][di][row comp][col comp]
                std::memset(E, 0, sizeof(E));
                double qq0[4], qr0[4], rr0[4];
                mapped_blocks(m, lam, mu, p, qq0, qr0, rr0);
                const int kind = (free_hi && j == nr) ? 1 : ((free_lo && j == 0) ? 2 : 0);
                if (kind != 0) {
                    // free row: q-compact as inside (weight 1/2, times 2); the
                    // r-edge into the domain; cross terms with the one-sided
                    // r difference (d = -1 top, +1 bottom)
                    const int d = kind == 1 ? -1 : 1;
                    for (int s = -1; s <= 1; s += 2) {
                        double qq[4], qr[4], rr[4];
                        mapped_blocks(m, lam, mu, p + s, qq, qr, rr);
                        for (int c = 0; c < 2; ++c)
                            for (int e = 0; e < 2; ++e) {
                                const double kb = 0.5 * (qq0[2 * c + e] + qq[2 * c + e]) * iqq;
                                E[1][1 + s][c][e] += kb;
                                E[1][1][c][e] -= kb;
                                // 2 x (1/2) D0q(K^qr Dhat_r U): K^qr at (j, i+s)
                                // times the one-sided r difference there
                                const double v = 2.0 * s * qr[2 * c + e] * iqr;
                                if (kind == 1) {   // (U_j - U_{j-1}) at i+s
                                    E[1][1 + s][c][e] += v;
                                    E[0][1 + s][c][e] -= v;
                                } else {           // (U_{j+1} - U_j) at i+s
                                    E[2][1 + s][c][e] += v;
                                    E[1][1 + s][c][e] -= v;
                                }
                            }
                    }
                    double qq[4], qr[4], rr[4];
                    mapped_blocks(m, lam, mu, p + d * sy, qq, qr, rr);   // the row inside
                    for (int c = 0; c < 2; ++c)
                        for (int e = 0; e < 2; ++e) {
                            const double kb = (rr0[2 * c + e] + rr[2 * c + e]) * irr;   // 2 x mean
                            E[1 + d][1][c][e] += kb;
                            E[1][1][c][e] -= kb;
                            // -/+ 2 (Q_row + Q_in) / (4 h_q h_r), Q = (K^qr)^T (U_{i+1} - U_{i-1})
                            const double sg = kind == 1 ? -2.0 * iqr : 2.0 * iqr;
                            E[1][2][c][e] += sg * qr0[2 * e + c];
                            E[1][0][c][e] -= sg * qr0[2 * e + c];
                            E[1 + d][2][c][e] += sg * qr[2 * e + c];
                            E[1 + d][0][c][e] -= sg * qr[2 * e + c];
                        }
                }
                for (int s = -1; s <= 1 && kind == 0; s += 2) {
                    double qq[4], qr[4], rr[4];
                    mapped_blocks(m, lam, mu, p + s, qq, qr, rr);   // (j, i+s)
                    for (int c = 0; c < 2; ++c)
                        for (int e = 0; e < 2; ++e) {
                            const double kb = 0.5 * (qq0[2 * c + e] + qq[2 * c + e]) * iqq;
                            E[1][1 + s][c][e] += kb;
                            E[1][1][c][e] -= kb;
                            // D0q(K^qr D0r U): K^qr at (j, i+s)
                            E[2][1 + s][c][e] += s * qr[2 * c + e] * iqr;
                            E[0][1 + s][c][e] -= s * qr[2 * c + e] * iqr;
                        }
                    mapped_blocks(m, lam, mu, p + s * sy, qq, qr, rr);   // (j+s, i)
                    for (int c = 0; c < 2; ++c)
                        for (int e = 0; e < 2; ++e) {
                            const double kb = 0.5 * (rr0[2 * c + e] + rr[2 * c + e]) * irr;
                            E[1 + s][1][c][e] += kb;
                            E[1][1][c][e] -= kb;
                            // D0r(K^rq D0q U): (K^qr)^T at (j+s, i)
                            E[1 + s][2][c][e] += s * qr[2 * e + c] * iqr;
                            E[1 + s][0][c][e] -= s * qr[2 * e + c] * iqr;
                        }
                }
                for (int c = 0; c < 2; ++c) {
                    double sum = 0.0;
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            const int jj = j + dj, ii = i + di;
                            if (jj < jlo || jj > jhi || ii < 1 || ii > nq - 1) continue;
                            sum += std::fabs(E[1 + dj][1 + di][c][0]) + std::fabs(E[1 + dj][1 + di][c][1]);
                        }
                    best = std::max(best, sum / (rho[p] * m.J[p]));   // free rows: entries carry the 2
                }
            }
        part[t] = best;
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nth; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& x : th) x.join();
    return *std::max_element(part.begin(), part.end());
}

// N_T, dt and c from the spectral bound G (shared by both grid kinds).
elwh_status plan_from_bound(double G, double omega, const elwh_opts* o, Plan* out, std::string* err) {
    const double T = 2.0 * M_PI / omega;
    int nt;
    if (o && o->nt > 0) {
        nt = o->nt;
    } else {
        const double cfl = o ? o->cfl : 0.8;
        const double dt_star = cfl * 2.0 / std::sqrt(G);
        const double q = std::ceil(T / dt_star);
        if (!(q < 1e8)) { *err = "too many steps per period"; return ELWH_ERR_ARG; }
        nt = std::max(3, (int)q);
    }
    if (o && o->scheme == ELWH_SCHEME_MODIFIED && nt < 4) {
        // the forcing frequency (2 / dt) asin(omega dt / 2) needs omega dt / 2 = pi / N_T < 1
        *err = "the modified trapezoid weights need at least 4 steps per period";
        return ELWH_ERR_ARG;
    }
    out->nt = nt;
    out->T = T;
    out->dt = T / nt;
    out->lambda_bound = G;
    // the standard and the modified-weights schemes step with the uncorrected leapfrog
    const bool corrected = !o || o->scheme == ELWH_SCHEME_CORRECTED;
    const double x = 0.5 * omega * out->dt;
    out->c = corrected ? (std::sin(x) / x) * (std::sin(x) / x) : 1.0;
    return ELWH_OK;
}

bool positive_materials(int64_t nn, const double* rho, const double* lam, const double* mu) {
    for (int64_t i = 0; i < nn; ++i)
        if (!(rho[i] > 0) || !(lam[i] > 0) || !(mu[i] > 0) || !std::isfinite(rho[i]) || !std::isfinite(lam[i]) ||
            !std::isfinite(mu[i]))
            return false;
    return true;
}

}  // namespace

// ---- discrete filter transfer function (App. B) --------------------------------

namespace {

// sum_{n=0}^{M} eta_n cos(n x), eta = 1/2 at both ends: sin(M x) / (2 tan(x / 2)),
// M at x = 0.
double trapezoid_cos_sum(int M, double x) {
    const double s = std::sin(0.5 * x);
    if (s == 0.0) return (double)M;
    return std::sin(M * x) * std::cos(0.5 * x) / (2.0 * s);
}

// beta_h at the rescaled frequency r (a mode cos(n theta), theta = r * 2 pi / N_T):
// sum_n w_n cos(n theta) with w_n = (2 / M) eta_n (cos(n phi) - 1/4), phi = 2 pi / N_T,
// M = K N_T, written with cos a cos b = (cos(a - b) + cos(a + b)) / 2.
double beta_rescaled(int nt, int periods, double r) {
    const int M = nt * periods;
    const double phi = 2.0 * M_PI / nt, th = r * phi;
    return (2.0 / M) * (0.5 * trapezoid_cos_sum(M, th - phi) + 0.5 * trapezoid_cos_sum(M, th + phi) -
                        0.25 * trapezoid_cos_sum(M, th));
}

}  // namespace

elwh_status filter_diagnostics(int nt, int periods, double omega, int scheme, elwh_filter_diag* out,
                               std::string* err) {
    if (!out) { *err = "null output"; return ELWH_ERR_ARG; }
    if (nt < 3) { *err = "nt must be >= 3"; return ELWH_ERR_ARG; }
    if (periods < 1 || periods > 1000) { *err = "periods must be in [1, 1000]"; return ELWH_ERR_ARG; }
    if (!(omega > 0) || !std::isfinite(omega)) { *err = "omega must be positive and finite"; return ELWH_ERR_ARG; }
    if (scheme != ELWH_SCHEME_CORRECTED && scheme != ELWH_SCHEME_STANDARD) { *err = "bad scheme"; return ELWH_ERR_ARG; }
    auto above = [&](double r) { return beta_rescaled(nt, periods, r) >= 1.0; };
    // increasing r: a linear scan of [1/2, 1 - 1e-3] and a logarithmic one of
    // 1 - 10^-3 .. 1 - 10^-15 (the band shrinks like dt^2); r = 1 itself, where
    // beta_h = 1 exactly, is left out.  The first sample at or above one and
    // the one before it bracket r*.
    std::vector<double> rs;
    for (int i = 0; i <= 20000; ++i) rs.push_back(0.5 + (0.5 - 1e-3) * i / 20000.0);
    for (int i = 1; i <= 1200; ++i) rs.push_back(1.0 - std::pow(10.0, -3.0 - 12.0 * i / 1200.0));
    double lo = -1, hi = -1;
    for (size_t i = 1; i < rs.size(); ++i)
        if (above(rs[i])) {
            if (above(rs[i - 1])) { *err = "transfer function at or above one below r = 1/2"; return ELWH_ERR_ARG; }
            lo = rs[i - 1];
            hi = rs[i];
            break;
        }
    if (hi < 0) {
        lo = hi = 1.0;   // no band above one that double precision resolves
    } else {
        for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
            const double mid = 0.5 * (lo + hi);
            (above(mid) ? hi : lo) = mid;
        }
    }
    out->r_star = hi;
    out->gap = 1.0 - hi;
    // maximum of beta_h over [r*, 1]: golden-section search (one peak)
    double a = hi, b = 1.0;
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
        const double c = b - g * (b - a), d = a + g * (b - a);
        if (beta_rescaled(nt, periods, c) >= beta_rescaled(nt, periods, d)) b = d; else a = c;
    }
    out->r_max = 0.5 * (a + b);
    out->beta_max = std::max(1.0, beta_rescaled(nt, periods, out->r_max));
    // spatial frequencies whose modes land in the band: theta = r omega dt with
    // sin(theta/2) = sin(omega dt/2) lambda / omega (corrected scheme) or
    // sin(theta/2) = lambda dt / 2 (standard scheme)
    const double dt = 2.0 * M_PI / omega / nt;
    auto lam = [&](double r) {
        const double th = r * omega * dt;
        return scheme == ELWH_SCHEME_CORRECTED ? omega * std::sin(0.5 * th) / std::sin(0.5 * omega * dt)
                                               : 2.0 * std::sin(0.5 * th) / dt;
    };
    out->lambda_lo = lam(out->r_star);
    out->lambda_hi = lam(1.0);
    return ELWH_OK;
}

elwh_status mapped_metric(int nq, int nr, const double* x, const double* y, MappedMetric* m, std::string* err) {
    const int64_t sy = nq + 1, nn = sy * (nr + 1);
    for (int64_t i = 0; i < nn; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i])) {
            *err = "node coordinates must be finite";
            return ELWH_ERR_ARG;
        }
    const double hq = 1.0 / nq, hr = 1.0 / nr;
    m->J.assign(nn, 0.0);
    for (auto& g : m->g) g.assign(nn, 0.0);
    for (int j = 0; j <= nr; ++j)
        for (int i = 0; i <= nq; ++i) {
            const int64_t o = j * sy + i;
            const double xq = diff1(x, o, 1, i, nq, hq), yq = diff1(y, o, 1, i, nq, hq);
            const double xr = diff1(x, o, sy, j, nr, hr), yr = diff1(y, o, sy, j, nr, hr);
            const double J = xq * yr - xr * yq;
            if (!(J > 0)) {
                *err = "the map must be one-to-one and orientation preserving (J > 0 at every node)";
                return ELWH_ERR_ARG;
            }
            m->J[o] = J;
            m->g[0][o] = yr;
            m->g[1][o] = -xr;
            m->g[2][o] = -yq;
            m->g[3][o] = xq;
        }
    return ELWH_OK;
}

elwh_status make_plan_mapped(const elwh_grid* g, const double* x, const double* y, const double* rho,
                             const double* lam, const double* mu, double omega, const int bc[6], const elwh_opts* o,
                             Plan* out, MappedMetric* met, std::string* err) {
    if (!g || !bc) { *err = "null grid or bc"; return ELWH_ERR_ARG; }
    if (g->dim != 2) { *err = "mapped grids are two-dimensional"; return ELWH_ERR_ARG; }
    if (bc[0] != ELWH_BC_DIRICHLET || bc[1] != ELWH_BC_DIRICHLET) {
        *err = "mapped grids need Dirichlet q sides (traction-free is supported on the r sides)";
        return ELWH_ERR_ARG;
    }
    elwh_grid unit = *g;
    unit.len[0] = unit.len[1] = 1.0;
    elwh_status st = check_config(&unit, bc, o, err);
    if (st != ELWH_OK) return st;
    if (!x || !y || !rho || !lam || !mu) { *err = "null coordinate or material array"; return ELWH_ERR_ARG; }
    if (!(omega > 0) || !std::isfinite(omega)) { *err = "omega must be positive and finite"; return ELWH_ERR_ARG; }
    const int nq = g->n[0], nr = g->n[1];
    if (!positive_materials((int64_t)(nq + 1) * (nr + 1), rho, lam, mu)) {
        *err = "materials must be positive and finite";
        return ELWH_ERR_ARG;
    }
    MappedMetric local;
    MappedMetric* m = met ? met : &local;
    if ((st = mapped_metric(nq, nr, x, y, m, err)) != ELWH_OK) return st;
    const double G = gershgorin_mapped(nq, nr, *m, rho, lam, mu, bc[2] == ELWH_BC_TRACTION_FREE,
                                       bc[3] == ELWH_BC_TRACTION_FREE);
    return plan_from_bound(G, omega, o, out, err);
}

// ---- mapped 3-D grids ---------------------------------------------------------

namespace {

// K^{ab} at node o, row-major 3x3: (lam/J) G_a G_b^T + (mu/J) (G_b G_a^T + (G_a . G_b) I).
void block3(const MappedMetric& m, const double* lam, const double* mu, int64_t o, int a, int b, double K[9]) {
    const double l = lam[o] / m.J[o], u = mu[o] / m.J[o];
    double ga[3], gb[3];
    for (int i = 0; i < 3; ++i) {
        ga[i] = m.g[3 * a + i][o];
        gb[i] = m.g[3 * b + i][o];
    }
    const double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) K[3 * i + k] = l * ga[i] * gb[k] + u * gb[i] * ga[k] + (i == k ? u * dot : 0.0);
}

// Entries of the node difference Dh along one axis at index t (0..N):
// central inside, one-sided into the domain on a free face, none on a
// Dirichlet face.  Returns the count; off[] are index offsets.
int dcoef(int t, int N, double h, bool free_lo, bool free_hi, int off[2], double cf[2]) {
    if (t >= 1 && t <= N - 1) {
        off[0] = 1; cf[0] = 0.5 / h;
        off[1] = -1; cf[1] = -0.5 / h;
        return 2;
    }
    if (t == 0 && free_lo) {
        off[0] = 1; cf[0] = 1.0 / h;
        off[1] = 0; cf[1] = -1.0 / h;
        return 2;
    }
    if (t == N && free_hi) {
        off[0] = 0; cf[0] = 1.0 / h;
        off[1] = -1; cf[1] = -1.0 / h;
        return 2;
    }
    return 0;
}

// Gershgorin row sums of (w_p rho J)^-1 L_h on a mapped 3-D grid, L_h = -grad
// of the energy E_h (edge terms with the mean K^aa of their two nodes,
// weight 1/2 for edges in a free s face; node terms w_n (Dh_a U)^T K^ab
// (Dh_b U) over ordered pairs a != b at unknown nodes): the 3x3 coefficient
// block of every neighbour of each unknown row, summed before taking
// absolute values, over unknown columns only.
double gershgorin_mapped3(int nq, int nr, int ns, const MappedMetric& m, const double* rho, const double* lam,
                          const double* mu, bool free_lo, bool free_hi) {
    const int N[3] = {nq, nr, ns};
    const double h[3] = {1.0 / nq, 1.0 / nr, 1.0 / ns};
    const int64_t st[3] = {1, (int64_t)nq + 1, (int64_t)(nq + 1) * (nr + 1)};
    const int klo = free_lo ? 0 : 1, khi = free_hi ? ns : ns - 1;
    auto unknown = [&](const int t[3]) {
        if (t[0] <= 0 || t[0] >= nq || t[1] <= 0 || t[1] >= nr) return false;
        return t[2] >= klo && t[2] <= khi;
    };
    auto wnode = [&](int k) { return ((k == 0 && free_lo) || (k == ns && free_hi)) ? 0.5 : 1.0; };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, (unsigned)std::max(1, khi - klo + 1));
    std::vector<double> part(nth, 0.0);
    auto work = [&](unsigned th) {
        double best = 0.0;
        double C[27][9];
        for (int k = klo + (int)th; k <= khi; k += (int)nth)
            for (int j = 1; j <= nr - 1; ++j)
                for (int i = 1; i <= nq - 1; ++i) {
                    const int tp[3] = {i, j, k};
                    const int64_t p = k * st[2] + j * st[1] + i;
                    std::memset(C, 0, sizeof(C));
                    auto cell = [](const int d[3]) { return (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1); };
                    double K0[9], K1[9];
                    // edge terms
                    for (int a = 0; a < 3; ++a) {
                        block3(m, lam, mu, p, a, a, K0);
                        for (int sg = -1; sg <= 1; sg += 2) {
                            const int t = tp[a] + sg;
                            if (t < 0 || t > N[a]) continue;
                            block3(m, lam, mu, p + sg * st[a], a, a, K1);
                            const double we = (a < 2 && ((k == 0 && free_lo) || (k == ns && free_hi))) ? 0.5 : 1.0;
                            int d[3] = {0, 0, 0};
                            d[a] = sg;
                            const double f = we * 0.5 / (h[a] * h[a]);
                            for (int e = 0; e < 9; ++e) {
                                C[cell(d)][e] += f * (K0[e] + K1[e]);
                                C[13][e] -= f * (K0[e] + K1[e]);
                            }
                        }
                    }
                    // node terms: -sum_n (Dh_a)_{n,p} w_n K^ab_n (Dh_b U)_n
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            if (a == b) continue;
                            for (int da = -1; da <= 1; ++da) {
                                int tn[3] = {i, j, k};
                                tn[a] += da;
                                if (!unknown(tn)) continue;
                                int oa[2], ob[2];
                                double ca[2], cb[2];
                                const int na = dcoef(tn[a], N[a], h[a], a == 2 && free_lo, a == 2 && free_hi, oa, ca);
                                double cpa = 0.0;
                                for (int q = 0; q < na; ++q)
                                    if (tn[a] + oa[q] == tp[a]) cpa += ca[q];
                                if (cpa == 0.0) continue;
                                const int64_t n = p + da * st[a];
                                const double wn = wnode(tn[2]);
                                double K[9];
                                block3(m, lam, mu, n, a, b, K);
                                const int nb = dcoef(tn[b], N[b], h[b], b == 2 && free_lo, b == 2 && free_hi, ob, cb);
                                for (int q = 0; q < nb; ++q) {
                                    int d[3] = {tn[0] - i, tn[1] - j, tn[2] - k};
                                    d[b] += ob[q];
                                    const double f = cpa * cb[q] * wn;
                                    for (int e = 0; e < 9; ++e) C[cell(d)][e] -= f * K[e];
                                }
                            }
                        }
                    const double scale = 1.0 / (rho[p] * m.J[p] * wnode(k));
                    for (int c = 0; c < 3; ++c) {
                        double row = 0.0;
                        for (int dz = -1; dz <= 1; ++dz)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int tm[3] = {i + dx, j + dy, k + dz};
                                    if (!unknown(tm)) continue;
                                    const int d[3] = {dx, dy, dz};
                                    for (int e = 0; e < 3; ++e) row += std::fabs(C[cell(d)][3 * c + e]);
                                }
                        best = std::max(best, row * scale);
                    }
                }
        part[th] = best;
    };
    std::vector<std::thread> thr;
    for (unsigned t = 1; t < nth; ++t) thr.emplace_back(work, t);
    work(0);
    for (auto& x : thr) x.join();
    return *std::max_element(part.begin(), part.end());
}

}  // namespace

elwh_status mapped_metric3(int nq, int nr, int ns, const double* x, const double* y, const double* z,
                           MappedMetric* m, std::string* err) {
    const int64_t sy = nq + 1, sz = sy * (nr + 1), nn = sz * (ns + 1);
    for (int64_t i = 0; i < nn; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i])) {
            *err = "node coordinates must be finite";
            return ELWH_ERR_ARG;
        }
    const double hq = 1.0 / nq, hr = 1.0 / nr, hs = 1.0 / ns;
    m->J.assign(nn, 0.0);
    for (auto& g : m->g) g.assign(nn, 0.0);
    const double* X[3] = {x, y, z};
    for (int k = 0; k <= ns; ++k)
        for (int j = 0; j <= nr; ++j)
            for (int i = 0; i <= nq; ++i) {
                const int64_t o = k * sz + j * sy + i;
                double dq[3], dr[3], ds[3];
                for (int c = 0; c < 3; ++c) {
                    dq[c] = diff1(X[c], o, 1, i, nq, hq);
                    dr[c] = diff1(X[c], o, sy, j, nr, hr);
                    ds[c] = diff1(X[c], o, sz, k, ns, hs);
                }
                auto cross = [](const double* a, const double* b, double* out) {
                    out[0] = a[1] * b[2] - a[2] * b[1];
                    out[1] = a[2] * b[0] - a[0] * b[2];
                    out[2] = a[0] * b[1] - a[1] * b[0];
                };
                double Gq[3], Gr[3], Gs[3];
                cross(dr, ds, Gq);
                cross(ds, dq, Gr);
                cross(dq, dr, Gs);
                const double J = dq[0] * Gq[0] + dq[1] * Gq[1] + dq[2] * Gq[2];
                if (!(J > 0)) {
                    *err = "the map must be one-to-one and orientation preserving (J > 0 at every node)";
                    return ELWH_ERR_ARG;
                }
                m->J[o] = J;
                for (int c = 0; c < 3; ++c) {
                    m->g[c][o] = Gq[c];
                    m->g[3 + c][o] = Gr[c];
                    m->g[6 + c][o] = Gs[c];
                }
            }
    return ELWH_OK;
}

elwh_status make_plan_mapped3(const elwh_grid* g, const double* x, const double* y, const double* z,
                              const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                              const elwh_opts* o, Plan* out, MappedMetric* met, std::string* err) {
    if (!g || !bc) { *err = "null grid or bc"; return ELWH_ERR_ARG; }
    if (g->dim != 3) { *err = "3-D mapped grids need dim = 3"; return ELWH_ERR_ARG; }
    for (int f = 0; f < 4; ++f)
        if (bc[f] != ELWH_BC_DIRICHLET) {
            *err = "3-D mapped grids need Dirichlet q and r faces (traction-free is supported on the s faces)";
            return ELWH_ERR_ARG;
        }
    elwh_grid unit = *g;
    unit.len[0] = unit.len[1] = unit.len[2] = 1.0;
    elwh_status st = check_config(&unit, bc, o, err);
    if (st != ELWH_OK) return st;
    if (!x || !y || !z || !rho || !lam || !mu) { *err = "null coordinate or material array"; return ELWH_ERR_ARG; }
    if (!(omega > 0) || !std::isfinite(omega)) { *err = "omega must be positive and finite"; return ELWH_ERR_ARG; }
    const int nq = g->n[0], nr = g->n[1], ns = g->n[2];
    if (!positive_materials((int64_t)(nq + 1) * (nr + 1) * (ns + 1), rho, lam, mu)) {
        *err = "materials must be positive and finite";
        return ELWH_ERR_ARG;
    }
    MappedMetric local;
    MappedMetric* m = met ? met : &local;
    if ((st = mapped_metric3(nq, nr, ns, x, y, z, m, err)) != ELWH_OK) return st;
    const double G = gershgorin_mapped3(nq, nr, ns, *m, rho, lam, mu, bc[4] == ELWH_BC_TRACTION_FREE,
                                        bc[5] == ELWH_BC_TRACTION_FREE);
    return plan_from_bound(G, omega, o, out, err);
}

elwh_status check_config(const elwh_grid* g, const int bc[6], const elwh_opts* o, std::string* err,
                         bool x_free_ok) {
    if (!g || !bc) { *err = "null grid or bc"; return ELWH_ERR_ARG; }
    if (g->dim != 2 && g->dim != 3) { *err = "dim must be 2 or 3"; return ELWH_ERR_ARG; }
    for (int a = 0; a < g->dim; ++a) {
        if (g->n[a] < 2) { *err = "need at least 2 cells per axis"; return ELWH_ERR_ARG; }
        if (g->n[a] > (1 << 20)) { *err = "grid too large"; return ELWH_ERR_ARG; }
        if (!(g->len[a] > 0) || !std::isfinite(g->len[a])) { *err = "box lengths must be positive"; return ELWH_ERR_ARG; }
    }
    for (int f = 0; f < 2 * g->dim; ++f)
        if (bc[f] != ELWH_BC_DIRICHLET && bc[f] != ELWH_BC_TRACTION_FREE) { *err = "bad boundary code"; return ELWH_ERR_ARG; }
    // traction-free faces only on the marching axis (y in 2-D, z in 3-D)
    const int march = g->dim - 1;
    for (int a = 0; a < g->dim; ++a)
        if (a != march && !(x_free_ok && g->dim == 2 && a == 0) &&
            (bc[2 * a] != ELWH_BC_DIRICHLET || bc[2 * a + 1] != ELWH_BC_DIRICHLET)) {
            *err = g->dim == 2 ? "traction-free faces are supported on the y faces only"
                               : "traction-free faces are supported on the z faces only";
            return ELWH_ERR_ARG;
        }
    if (o) {
        if (!(o->cfl > 0) || !(o->cfl < 1.0 + 1e-12)) { *err = "cfl must be in (0, 1]"; return ELWH_ERR_ARG; }
        if (o->nt < 0 || (o->nt > 0 && o->nt < 3)) { *err = "nt must be 0 (rule) or >= 3"; return ELWH_ERR_ARG; }
        if (o->periods < 1 || o->periods > 1000) { *err = "periods must be in [1, 1000]"; return ELWH_ERR_ARG; }
        if (o->prec != ELWH_FP64 && o->prec != ELWH_FP32_STEP) { *err = "bad precision"; return ELWH_ERR_ARG; }
        if (o->krylov < 0 || o->krylov > 3) { *err = "bad krylov method"; return ELWH_ERR_ARG; }
        if (o->cr_fallback < 0 || o->cr_fallback > 2) { *err = "cr_fallback must be 0, 1 or 2"; return ELWH_ERR_ARG; }
        if (o->prec == ELWH_FP32_STEP && o->krylov != ELWH_KRYLOV_CG) {
            *err = "FP32 stepping solves with CG (residual-replacement segments); GMRES, CR and MINRES need FP64";
            return ELWH_ERR_ARG;
        }
        if (o->gmres_m < 1 || o->gmres_m > 200) { *err = "gmres_m must be in [1, 200]"; return ELWH_ERR_ARG; }
        if (o->scheme != ELWH_SCHEME_CORRECTED && o->scheme != ELWH_SCHEME_STANDARD &&
            o->scheme != ELWH_SCHEME_MODIFIED) { *err = "bad scheme"; return ELWH_ERR_ARG; }
        if (o->fuse < 1 || o->fuse > 4) { *err = "fuse must be in [1, 4]"; return ELWH_ERR_ARG; }
        if (!(o->fp32_switch >= 0.0 && o->fp32_switch < 1.0)) {
            *err = "fp32_switch must be in [0, 1)";
            return ELWH_ERR_ARG;
        }
    }
    return ELWH_OK;
}

elwh_status make_plan(const elwh_grid* g, const double* rho, const double* lam, const double* mu,
                      double omega, const int bc[6], const elwh_opts* o, Plan* out, std::string* err,
                      bool x_free_ok) {
    elwh_status st = check_config(g, bc, o, err, x_free_ok);
    if (st != ELWH_OK) return st;
    if (!rho || !lam || !mu) { *err = "null material array"; return ELWH_ERR_ARG; }
    if (!(omega > 0) || !std::isfinite(omega)) { *err = "omega must be positive and finite"; return ELWH_ERR_ARG; }
    Geo geo;
    geo.d = g->dim;
    for (int a = 0; a < 3; ++a) {
        geo.n[a] = a < g->dim ? g->n[a] : 0;
        geo.h[a] = a < g->dim ? g->len[a] / g->n[a] : 1.0;
    }
    for (int f = 0; f < 6; ++f) geo.bc[f] = f < 2 * g->dim ? bc[f] : ELWH_BC_DIRICHLET;
    geo.sx = 1;
    geo.sy = g->n[0] + 1;
    geo.sz = (int64_t)(g->n[0] + 1) * (g->n[1] + 1);
    geo.rho = rho;
    geo.lam = lam;
    geo.mu = mu;
    const int64_t nn = geo.sz * (g->dim == 3 ? g->n[2] + 1 : 1);
    if (!positive_materials(nn, rho, lam, mu)) {
        *err = "materials must be positive and finite";
        return ELWH_ERR_ARG;
    }
    return plan_from_bound(gershgorin(geo), omega, o, out, err);
}

Layout make_layout(const elwh_grid* g) {
    Layout L;
    L.dim = g->dim;
    L.nx = g->n[0];
    L.ny = g->n[1];
    L.nz = g->dim == 3 ? g->n[2] : 0;
    // at least 3 padding elements, so a 4-wide vector starting at any node
    // column stays inside its row
    L.P = ((int64_t)(L.nx + 4) + 63) / 64 * 64;
    L.PS = (int64_t)(L.ny + 1) * L.P;
    L.CS = L.PS * (L.dim == 3 ? (L.nz + 1) : 1);
    return L;
}

Stencil make_stencil(const elwh_grid* g) {
    Stencil s;
    const double hx = g->len[0] / g->n[0], hy = g->len[1] / g->n[1];
    const double hz = g->dim == 3 ? g->len[2] / g->n[2] : 1.0;
    s.cxx2 = 0.5 / (hx * hx);
    s.cyy2 = 0.5 / (hy * hy);
    s.czz2 = 0.5 / (hz * hz);
    s.cxy = 0.25 / (hx * hy);
    s.cxz = 0.25 / (hx * hz);
    s.cyz = 0.25 / (hy * hz);
    s.cyyf = 1.0 / (hy * hy);
    s.czzf = 1.0 / (hz * hz);
    s.cfxy = 0.5 / (hx * hy);
    s.cfxz = 0.5 / (hx * hz);
    s.cfyz = 0.5 / (hy * hz);
    return s;
}

March make_march(const elwh_grid* g, const int bc[6]) {
    March m;
    const int a = g->dim - 1;
    m.free_lo = bc[2 * a] == ELWH_BC_TRACTION_FREE;
    m.free_hi = bc[2 * a + 1] == ELWH_BC_TRACTION_FREE;
    m.lo = m.free_lo ? 0 : 1;
    m.hi = m.free_hi ? g->n[a] : g->n[a] - 1;
    return m;
}

}  // namespace elwh
