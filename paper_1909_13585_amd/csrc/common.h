// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlb {

// Element-local node a = bx + 2*by + 4*bz (offset of the node from the
// element's lowest corner); local DOF = dim*a + c.
constexpr int nn_of(int dim) { return 1 << dim; }
constexpr int nde_of(int dim) { return dim << dim; }
constexpr int nv_of(int dim) { return dim == 2 ? 3 : 6; }

constexpr int kBlock = 256;          // threads per block for 1D kernels
constexpr int kMaxPartials = 1024;   // blocks per reduction stage
// fixed device scratch of the no-allocation entry points (scratch.hip):
// per-block partial maxima and the maxima of up to kNoallocMaxSel rows
constexpr int kNoallocMaxSel = 64;
constexpr int64_t kScratchDoubles = (int64_t)kMaxPartials * kNoallocMaxSel + kNoallocMaxSel;

// Geometry of one grid level (unit elements at level 1).
struct Geo {
    int nx, ny, nz;          // elements per axis (nz = 1 for 2D)
    int nnx, nny, nnz;       // nodes per axis (nnz = 1 for 2D)
    int64_t m;               // elements
    int64_t nodes;           // nodes
};

inline Geo make_geo(int dim, const int* nel) {
    Geo g;
    g.nx = nel[0];
    g.ny = nel[1];
    g.nz = dim == 3 ? nel[2] : 1;
    g.nnx = g.nx + 1;
    g.nny = g.ny + 1;
    g.nnz = dim == 3 ? g.nz + 1 : 1;
    g.m = (int64_t)g.nx * g.ny * g.nz;
    g.nodes = (int64_t)g.nnx * g.nny * g.nnz;
    return g;
}

// Apply-kernel epilogues.
enum ApplyMode { kModeY = 0, kModeResidual = 1, kModeJacobi = 2 };

}  // namespace mlb
