// Element and transfer tables of the Q4/H8 discretisation (host, FP64).
//
// Sec. 2: K_e = E_kappa(x_e) K_e0 and G_e = E_sigma(x_e) G_e0[u_e].  The
// element is the bilinear (2D, plane stress, unit thickness) or trilinear
// (3D) unit square/cube; K_e0 = integral B^T D0 B with 2 Gauss points per
// axis (exact for these elements); G_e0 uses one stress per element, at the
// centroid: G_e0 = (sum_ij sigma_ij H^ij) kron I_dim, H^ij = integral of
// dN/dx_i dN/dx_j^T.  With element == 1 (the paper's incompatible Q6/H11,
// Sec. 2) every displacement component gets one mode 4 x_m (1 - x_m) per
// axis, condensed out of K_e0; their gradients vanish at the centroid, so
// the centroid stress and G_e0 are those of the nodal interpolation.  Voigt order: 2D (xx, yy, xy), 3D (xx, yy, zz, xy, yz,
// xz), engineering shear strains.
//
// Galerkin coarsening (Sec. 2.1 step 1): a coarse element of level j+1 holds
// 2^dim children of level j; child c = cx + 2cy + 4cz.  The child's local
// node b sits at lattice point c + b (0..2 per axis) of the coarse element,
// where nodal interpolation gives coarse node A the weight
//   w = prod_axis w1(p, A),  w1(0,0) = w1(2,1) = 1, w1(1,*) = 1/2, else 0.
// T[c][b][A] stores it; then K_E = sum_c T_c^T K_c T_c (kron I for vectors).
#include "tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace mlb {

static double shape(int dim, int a, const double* xi) {
    double v = 1.0;
    for (int k = 0; k < dim; ++k) {
        int b = (a >> k) & 1;
        v *= b ? xi[k] : 1.0 - xi[k];
    }
    return v;
}

static double shape_grad(int dim, int a, int i, const double* xi) {
    double v = 1.0;
    for (int k = 0; k < dim; ++k) {
        int b = (a >> k) & 1;
        if (k == i) v *= b ? 1.0 : -1.0;
        else v *= b ? xi[k] : 1.0 - xi[k];
    }
    return v;
}

// Strain-displacement matrix at xi: rows Voigt strains, cols dim*a + c.
static void strain_disp(int dim, const double* xi, double* B /* nv x nde */) {
    const int nn = 1 << dim, nde = dim * nn, nv = dim == 2 ? 3 : 6;
    std::memset(B, 0, sizeof(double) * nv * nde);
    for (int a = 0; a < nn; ++a) {
        double g[3];
        for (int i = 0; i < dim; ++i) g[i] = shape_grad(dim, a, i, xi);
        if (dim == 2) {
            B[0 * nde + 2 * a + 0] = g[0];
            B[1 * nde + 2 * a + 1] = g[1];
            B[2 * nde + 2 * a + 0] = g[1];
            B[2 * nde + 2 * a + 1] = g[0];
        } else {
            B[0 * nde + 3 * a + 0] = g[0];
            B[1 * nde + 3 * a + 1] = g[1];
            B[2 * nde + 3 * a + 2] = g[2];
            B[3 * nde + 3 * a + 0] = g[1];  // gamma_xy
            B[3 * nde + 3 * a + 1] = g[0];
            B[4 * nde + 3 * a + 1] = g[2];  // gamma_yz
            B[4 * nde + 3 * a + 2] = g[1];
            B[5 * nde + 3 * a + 0] = g[2];  // gamma_xz
            B[5 * nde + 3 * a + 2] = g[0];
        }
    }
}

// Strains of the incompatible modes at xi (nv x dim^2): column dim*c + m is
// the field u_c = 4 x_m (1 - x_m), zero at the nodes, whose only nonzero
// derivative is d u_c / d x_m = 4 - 8 x_m.
static void bubble_strain(int dim, const double* xi, double* Bt) {
    const int nv = dim == 2 ? 3 : 6, ni = dim * dim;
    std::memset(Bt, 0, sizeof(double) * nv * ni);
    static const int shear3[3][2] = {{0, 1}, {1, 2}, {0, 2}};   // Voigt rows 3, 4, 5
    for (int c = 0; c < dim; ++c)
        for (int m = 0; m < dim; ++m) {
            const double g = 4.0 - 8.0 * xi[m];
            const int col = dim * c + m;
            if (m == c) Bt[c * ni + col] = g;                  // normal strain
            if (dim == 2) {
                if (m != c) Bt[2 * ni + col] = g;              // gamma_xy
            } else {
                for (int r = 0; r < 3; ++r) {
                    const int i = shear3[r][0], j = shear3[r][1];
                    if ((c == i && m == j) || (c == j && m == i)) Bt[(3 + r) * ni + col] = g;
                }
            }
        }
}

static double interp_w1(int p, int A) {
    if (p == 1) return 0.5;
    if (p == 0) return A == 0 ? 1.0 : 0.0;
    return A == 1 ? 1.0 : 0.0;  // p == 2
}

void build_tables(int dim, double nu, int element, Tables* t) {
    std::memset(t, 0, sizeof(Tables));
    t->dim = dim;
    const int nn = 1 << dim, nde = dim * nn, nv = dim == 2 ? 3 : 6;
    t->nn = nn;
    t->nde = nde;
    t->nv = nv;

    // unit-modulus constitutive matrix
    if (dim == 2) {
        const double s = 1.0 / (1.0 - nu * nu);
        double D[9] = {s, s * nu, 0, s * nu, s, 0, 0, 0, s * (1.0 - nu) / 2.0};
        std::memcpy(t->D0, D, sizeof(D));
    } else {
        const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double mu = 1.0 / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) t->D0[i * 6 + j] = lam + (i == j ? 2.0 * mu : 0.0);
        for (int i = 3; i < 6; ++i) t->D0[i * 6 + i] = mu;
    }

    // Gauss points on [0,1]
    const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    const int ngp = 1 << dim;
    const double wgp = 1.0 / ngp;
    double B[6 * 24], DB[6 * 24];
    double Hij[3][3][64];
    std::memset(Hij, 0, sizeof(Hij));
    // incompatible modes: couplings K_ci (nde x ni) and K_ii (ni x ni)
    const int ni = dim * dim;
    double Bt[6 * 9], Kci[24 * 9], Kii[9 * 9];
    std::memset(Kci, 0, sizeof(Kci));
    std::memset(Kii, 0, sizeof(Kii));
    for (int q = 0; q < ngp; ++q) {
        double xi[3];
        for (int k = 0; k < dim; ++k) xi[k] = gp[(q >> k) & 1];
        strain_disp(dim, xi, B);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nde; ++j) {
                double s = 0;
                for (int k = 0; k < nv; ++k) s += t->D0[i * nv + k] * B[k * nde + j];
                DB[i * nde + j] = s;
            }
        for (int i = 0; i < nde; ++i)
            for (int j = 0; j < nde; ++j) {
                double s = 0;
                for (int k = 0; k < nv; ++k) s += B[k * nde + i] * DB[k * nde + j];
                t->K0[i * nde + j] += wgp * s;
            }
        if (element == 1) {
            bubble_strain(dim, xi, Bt);
            for (int i = 0; i < ni; ++i) {
                double DBt[6];
                for (int k = 0; k < nv; ++k) {
                    double s = 0;
                    for (int l = 0; l < nv; ++l) s += t->D0[k * nv + l] * Bt[l * ni + i];
                    DBt[k] = s;
                }
                for (int a = 0; a < nde; ++a) {
                    double s = 0;
                    for (int k = 0; k < nv; ++k) s += B[k * nde + a] * DBt[k];
                    Kci[a * ni + i] += wgp * s;
                }
                for (int j = 0; j < ni; ++j) {
                    double s = 0;
                    for (int k = 0; k < nv; ++k) s += Bt[k * ni + j] * DBt[k];
                    Kii[j * ni + i] += wgp * s;
                }
            }
        }
        double g[8][3];
        for (int a = 0; a < nn; ++a)
            for (int i = 0; i < dim; ++i) g[a][i] = shape_grad(dim, a, i, xi);
        for (int i = 0; i < dim; ++i)
            for (int j = 0; j < dim; ++j)
                for (int a = 0; a < nn; ++a)
                    for (int b = 0; b < nn; ++b) Hij[i][j][a * nn + b] += wgp * g[a][i] * g[b][j];
    }
    // static condensation of the incompatible modes: K0 -= K_ci K_ii^-1 K_ci^T
    // (K_ii is SPD: Cholesky, then one solve per nodal DOF)
    if (element == 1) {
        double L[81];
        std::memcpy(L, Kii, sizeof(double) * ni * ni);
        for (int j = 0; j < ni; ++j) {
            double d = L[j * ni + j];
            for (int k = 0; k < j; ++k) d -= L[j * ni + k] * L[j * ni + k];
            L[j * ni + j] = std::sqrt(d);
            for (int i = j + 1; i < ni; ++i) {
                double s = L[i * ni + j];
                for (int k = 0; k < j; ++k) s -= L[i * ni + k] * L[j * ni + k];
                L[i * ni + j] = s / L[j * ni + j];
            }
        }
        std::vector<double> Y((size_t)nde * ni);   // Y = K_ii^-1 K_ci^T, column per nodal DOF
        for (int a = 0; a < nde; ++a) {
            double y[9];
            for (int i = 0; i < ni; ++i) {
                double s = Kci[a * ni + i];
                for (int k = 0; k < i; ++k) s -= L[i * ni + k] * y[k];
                y[i] = s / L[i * ni + i];
            }
            for (int i = ni - 1; i >= 0; --i) {
                double s = y[i];
                for (int k = i + 1; k < ni; ++k) s -= L[k * ni + i] * y[k];
                y[i] = s / L[i * ni + i];
            }
            for (int i = 0; i < ni; ++i) Y[(size_t)a * ni + i] = y[i];
        }
        for (int a = 0; a < nde; ++a)
            for (int b = 0; b < nde; ++b) {
                double s = 0;
                for (int i = 0; i < ni; ++i) s += Kci[a * ni + i] * Y[(size_t)b * ni + i];
                t->K0[a * nde + b] -= s;
            }
    }
    // symmetrise K0 exactly
    for (int i = 0; i < nde; ++i)
        for (int j = 0; j < i; ++j) {
            double v = 0.5 * (t->K0[i * nde + j] + t->K0[j * nde + i]);
            t->K0[i * nde + j] = t->K0[j * nde + i] = v;
        }
    // Voigt-combined gradient products: normal H^ii, shear H^ij + H^ji
    static const int pairs2[3][2] = {{0, 0}, {1, 1}, {0, 1}};
    static const int pairs3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {0, 2}};
    for (int k = 0; k < nv; ++k) {
        int i = dim == 2 ? pairs2[k][0] : pairs3[k][0];
        int j = dim == 2 ? pairs2[k][1] : pairs3[k][1];
        for (int ab = 0; ab < nn * nn; ++ab)
            t->Hk[k * 64 + ab] = (i == j) ? Hij[i][i][ab] : Hij[i][j][ab] + Hij[j][i][ab];
    }
    // centroid strain matrix and D0 * Bc
    double xc[3] = {0.5, 0.5, 0.5};
    strain_disp(dim, xc, B);
    for (int i = 0; i < nv * nde; ++i) t->Bc[i] = B[i];
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nde; ++j) {
            double s = 0;
            for (int k = 0; k < nv; ++k) s += t->D0[i * nv + k] * B[k * nde + j];
            t->D0Bc[i * nde + j] = s;
        }

    // child interpolation weights T[c][b][A]
    const int nch = 1 << dim;
    for (int c = 0; c < nch; ++c)
        for (int b = 0; b < nn; ++b)
            for (int A = 0; A < nn; ++A) {
                double w = 1.0;
                for (int k = 0; k < dim; ++k) {
                    int p = ((c >> k) & 1) + ((b >> k) & 1);
                    w *= interp_w1(p, (A >> k) & 1);
                }
                t->T[(c * 8 + b) * 8 + A] = w;
            }
    // Mc = T_c^T K0 T_c (vector form) and GHc_k = T_c^T H^k T_c (scalar form)
    for (int c = 0; c < nch; ++c) {
        for (int A = 0; A < nn; ++A)
            for (int ca = 0; ca < dim; ++ca)
                for (int Bn = 0; Bn < nn; ++Bn)
                    for (int cb = 0; cb < dim; ++cb) {
                        double s = 0;
                        for (int b = 0; b < nn; ++b) {
                            double wa = t->T[(c * 8 + b) * 8 + A];
                            if (wa == 0.0) continue;
                            for (int b2 = 0; b2 < nn; ++b2) {
                                double wb = t->T[(c * 8 + b2) * 8 + Bn];
                                if (wb == 0.0) continue;
                                s += wa * wb * t->K0[(b * dim + ca) * nde + b2 * dim + cb];
                            }
                        }
                        t->Mc[(size_t)c * 576 + (A * dim + ca) * nde + Bn * dim + cb] = s;
                    }
        for (int k = 0; k < nv; ++k)
            for (int A = 0; A < nn; ++A)
                for (int Bn = 0; Bn < nn; ++Bn) {
                    double s = 0;
                    for (int b = 0; b < nn; ++b)
                        for (int b2 = 0; b2 < nn; ++b2)
                            s += t->T[(c * 8 + b) * 8 + A] * t->T[(c * 8 + b2) * 8 + Bn] *
                                 t->Hk[k * 64 + b * nn + b2];
                    t->GHc[((size_t)c * 6 + k) * 64 + A * nn + Bn] = s;
                }
    }

    // Symmetry-adapted Walsh-Hadamard blocks: D = (Hb kron I) K0 (Hb kron I)
    // with Hb[k][a] = (-1)^popcount(k & a); component c of block sigma sits at
    // transform index sigma ^ (1 << c).  K0 = H D H / 4^dim.
    auto hb = [](int k, int a) { return (__builtin_popcount(k & a) & 1) ? -1.0 : 1.0; };
    std::vector<double> D((size_t)nde * nde, 0.0);
    for (int k = 0; k < nn; ++k)
        for (int c = 0; c < dim; ++c)
            for (int k2 = 0; k2 < nn; ++k2)
                for (int c2 = 0; c2 < dim; ++c2) {
                    double s = 0;
                    for (int a = 0; a < nn; ++a)
                        for (int b = 0; b < nn; ++b)
                            s += hb(k, a) * t->K0[(a * dim + c) * nde + b * dim + c2] * hb(k2, b);
                    D[(size_t)(k * dim + c) * nde + k2 * dim + c2] = s;
                }
    double dmax = 0, offmax = 0;
    for (double v : D) dmax = std::max(dmax, std::fabs(v));
    const double scale = 1.0 / (double)(nn * nn);
    for (int row = 0; row < nde; ++row)
        for (int colm = 0; colm < nde; ++colm) {
            const int k = row / dim, c = row % dim, k2 = colm / dim, c2 = colm % dim;
            const int s1 = k ^ (1 << c), s2 = k2 ^ (1 << c2);
            // structural pattern: translation rows/columns vanish, components
            // c != c2 couple only where bits c and c2 of the block index agree
            const bool nz = s1 == s2 && s1 != (1 << c) && s1 != (1 << c2) && (((s1 >> c) & 1) == ((s1 >> c2) & 1));
            if (!nz) offmax = std::max(offmax, std::fabs(D[(size_t)row * nde + colm]));
            if (s1 == s2) t->wht[s1 * dim * dim + c * dim + c2] = nz ? D[(size_t)row * nde + colm] * scale : 0.0;
        }
    // The unit square/cube with an isotropic material is also invariant under
    // axis permutations, which ties the blocks to a few numbers:
    //   3D: B_0 = d0 I + o0 (J - I), B_7 = d7 I + o7 (J - I); for sigma = 1<<c
    //   the two other components form [[e1, f1], [f1, e1]]; for sigma with two
    //   bits set those components form [[g2d, g2o], [g2o, g2d]] and the third
    //   has h2.  2D: B_0 = [[d0, o0], [o0, d0]], one-bit blocks q1, B_3 =
    //   [[d3, o3], [o3, d3]].  The kernel uses these numbers; check that they
    //   reproduce every block exactly.
    double rec[72] = {};
    if (dim == 3) {
        const double* w = t->wht;
        double* v = t->whs;
        v[0] = w[0];          v[1] = w[1];            // d0, o0
        v[2] = w[7 * 9 + 0];  v[3] = w[7 * 9 + 1];    // d7, o7
        v[4] = w[1 * 9 + 4];  v[5] = w[1 * 9 + 5];    // e1, f1
        v[6] = w[3 * 9 + 0];  v[7] = w[3 * 9 + 1];    // g2d, g2o
        v[8] = w[3 * 9 + 8];                          // h2
        for (int sg = 0; sg < 8; ++sg)
            for (int c = 0; c < 3; ++c)
                for (int c2 = 0; c2 < 3; ++c2) {
                    const int bits = __builtin_popcount(sg);
                    double r = 0.0;
                    if (bits == 0) r = c == c2 ? v[0] : v[1];
                    else if (bits == 3) r = c == c2 ? v[2] : v[3];
                    else if (bits == 1) {
                        if (((sg >> c) & 1) == 0 && ((sg >> c2) & 1) == 0) r = c == c2 ? v[4] : v[5];
                    } else {
                        const bool in1 = (sg >> c) & 1, in2 = (sg >> c2) & 1;
                        if (in1 && in2) r = c == c2 ? v[6] : v[7];
                        else if (!in1 && !in2 && c == c2) r = v[8];
                    }
                    rec[sg * 9 + c * 3 + c2] = r;
                }
    } else {
        const double* w = t->wht;
        double* v = t->whs;
        v[0] = w[0];          v[1] = w[1];            // d0, o0
        v[2] = w[1 * 4 + 3];                          // q1
        v[3] = w[3 * 4 + 0];  v[4] = w[3 * 4 + 1];    // d3, o3
        for (int sg = 0; sg < 4; ++sg)
            for (int c = 0; c < 2; ++c)
                for (int c2 = 0; c2 < 2; ++c2) {
                    double r = 0.0;
                    if (sg == 0) r = c == c2 ? v[0] : v[1];
                    else if (sg == 3) r = c == c2 ? v[3] : v[4];
                    else if (c == c2 && ((sg >> c) & 1) == 0) r = v[2];
                    rec[sg * 4 + c * 2 + c2] = r;
                }
    }
    double symdiff = 0.0;
    for (int i = 0; i < nn * dim * dim; ++i) symdiff = std::max(symdiff, std::fabs(rec[i] - t->wht[i]));
    t->wht_ok = offmax <= 1e-13 * dmax && symdiff <= 1e-13 * dmax;
}

}  // namespace mlb
