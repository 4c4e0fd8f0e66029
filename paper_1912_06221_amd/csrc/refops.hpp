// Host-side FP64 construction of the reference operators of order N.
#pragma once

#include <vector>

#include "dense.hpp"

namespace ardg {

// Index of lattice point (i, j) (i along r, j along s, i + j <= N) in the
// row-by-row node order.
inline int lattice_index(int N, int i, int j) {
  return j * (N + 1) - (j * (j - 1)) / 2 + i;
}

struct RefOps {
  int N = 0, Np = 0, Nfp = 0, Mp = 0;
  std::vector<double> r, s;          // node coordinates
  std::vector<double> lgl;           // 1D LGL points, increasing
  Mat V, Vinv, Dr, Ds, M, Minv, LIFT;
  int fmask[3][16];                  // face node indices, CCW
  int rot[3][64];                    // (Pi_f u)_i = u[rot[f][i]]
  Mat Bv, N2B, B2psi;                // Bernstein at nodes, its inverse, Bernstein -> modal
  Mat A, Rop;                        // least-squares system and its pseudo-inverse
  double recon_cond = 0.0;
  // Constant per-edge operators acting on Bernstein coefficients of the two
  // sub-triangles ([c1; c2], each in its own frame):
  Mat KR, KS;                        // (d/dR, d/dS) u~ at the diagonal nodes [Nfp][2Np]
  Mat U1R, U1S, U2R, U2S;            // Algorithm 1 blocks [Nfp][2Np]
  Mat KBR, KBS;                      // boundary (mirror ghost) versions [Nfp][Np]
  Mat UBR, UBS;                      // Algorithm 1 boundary versions [Nfp][Np]
  // Algorithm 2: the reconstruction of a coefficient that is 1 on one
  // sub-triangle and 0 on the other, at the diagonal nodes, so that an
  // element-wise constant coefficient reconstructs to D1 w1 + D2 w2 there.
  std::vector<double> alg2_w1, alg2_w2;   // [Nfp]
  // Algorithm 1 with a nodal coefficient: the reference gradient (d/dr,
  // d/ds in each sub-triangle's own frame) of u~ at the nodes of sub-triangle
  // k from the Bernstein coefficients of both sub-triangles [Np][2Np], and the
  // map from nodal data on sub-triangle k to values at the diagonal nodes
  // (the second reconstruction) [Nfp][Np].
  Mat TR1, TS1, TR2, TS2, G1, G2;
  // Values of u~ at the diagonal nodes from the Bernstein coefficients of
  // both sub-triangles [Nfp][2Np] (the Navier-Stokes interface needs the
  // reconstructed temperature and velocity, not only their gradients).
  Mat KV;
  // The same maps on nodal sub-triangle data (for export / checking).
  Mat recon_grad_nodal;              // [2Nfp][2Np]
  Mat alg1_nodal;                    // [4Nfp][2Np]
  Mat recon_value_nodal;             // [Nfp][2Np]
};

// Throws std::runtime_error on failure; sets *rank_ok false if the
// reconstruction system is rank deficient.
RefOps build_refops(int N, bool* rank_ok);

// 1D helpers (also used by the mesh setup).
std::vector<double> lgl_points(int N);
double jacobi_p(double x, int n, double alpha, double beta);

}  // namespace ardg
