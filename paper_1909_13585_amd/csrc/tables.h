// Host-built element and transfer tables (FP64), uploaded once per context.
#pragma once

namespace mlb {

struct Tables {
    int dim, nn, nde, nv;
    double D0[36];          // nv x nv unit-modulus constitutive matrix
    double K0[576];         // nde x nde unit-modulus element stiffness
    double Hk[6 * 64];      // nv x (nn x nn) Voigt-combined gradient products
    double Bc[6 * 24];      // nv x nde centroid strain matrix
    double D0Bc[6 * 24];    // nv x nde, D0 * Bc
    double T[8 * 8 * 8];    // child c, child node b, coarse node A -> weight
    double Mc[8 * 576];     // child c: T_c^T K0 T_c (nde x nde)
    double GHc[8 * 6 * 64]; // child c, Voigt k: T_c^T H^k T_c (nn x nn)
    double wht[8 * 9];      // symmetry-adapted Walsh-Hadamard blocks of K0 / 4^dim
    double whs[9];          // the few numbers those blocks are made of (see tables.cpp)
    bool wht_ok;            // K0 is exactly block diagonal in that basis, with that structure
};

// element: 0 bilinear/trilinear, 1 with condensed incompatible modes
void build_tables(int dim, double nu, int element, Tables* t);

}  // namespace mlb
