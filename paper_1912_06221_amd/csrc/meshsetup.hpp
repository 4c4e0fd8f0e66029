// Host-side FP64 mesh setup: connectivity, enclosed parallelograms and the
// per-edge parameters the kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ardg {

struct HostMesh {
  int64_t K = 0, Nv = 0, E_int = 0, E_bdy = 0;
  std::vector<double> vxy;                 // [Nv][2]
  std::vector<int32_t> etov;               // [K][3]
  std::vector<double> J;                   // [K]
  // interior edges, side 1 = lower element index
  std::vector<int32_t> e1, f1, e2, f2;     // [E_int]
  std::vector<double> P1;                  // [E_int][2] parallelogram apex in element 1
  std::vector<double> mu1, mu2;            // [E_int][2] (lambda_w2, lambda_w3) of P_k in
                                           // element k's rotated frame
  std::vector<double> gam;                 // [E_int][2] gamma_R, gamma_S
  // boundary faces
  std::vector<int32_t> bk, bf;             // [E_bdy]
  std::vector<double> bP1, bmu, bgam;      // [E_bdy][2]
  std::vector<int32_t> elem_face;          // [K][3] (edge << 1) | side
  double min_J = 0.0, min_area_ratio = 1.0;
};

// Returns 0 on success or a negative ardg status with a message in err.
int build_host_mesh(const double* vxy, int64_t Nv, const int32_t* etov, int64_t K,
                    HostMesh& m, std::string& err);

}  // namespace ardg
