// Device-side mesh description and kernel launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ardg {

constexpr int kMaxFields = 16;

// Arithmetic of the operator products (values as in the C ABI).  FP64:
// double data; FP32: float data; BF16X3: float data, products on the BF16
// matrix cores with split operands (hi + lo) and FP32 accumulation.
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

// Offsets of the packed constant operators (same layout in FP64 and FP32).
// bf2n: 1D Bernstein coefficients of a face -> values at its LGL nodes;
// w1, w2: Algorithm 2's diagonal weights of the two sides' coefficients;
// tr1, ts1, tr2, ts2, g1, g2: Algorithm 1 with a nodal coefficient (reference
// gradients of u~ at each sub-triangle's nodes from both sides' Bernstein
// coefficients, nodal data on a sub-triangle -> diagonal values); b2n:
// Bernstein coefficients -> nodal values; kv: values of u~ at the diagonal
// nodes from both sides' Bernstein coefficients.
struct OpLayout {
  int Np, Nfp;
  int n2b, kr, ks, kbr, kbs, u1r, u1s, u2r, u2s, udr, uds, ubr, ubs, dr, ds, drsh, lift, tau, nr, ns;
  int bf2n, w1, w2, tr1, ts1, tr2, ts2, g1, g2, b2n, kv, total;
  __host__ __device__ constexpr OpLayout(int N)
      : Np((N + 1) * (N + 2) / 2), Nfp(N + 1),
        n2b(0),
        kr(Np * Np),
        ks(kr + Nfp * 2 * Np),
        kbr(ks + Nfp * 2 * Np),
        kbs(kbr + Nfp * Np),
        u1r(kbs + Nfp * Np),
        u1s(u1r + Nfp * 2 * Np),
        u2r(u1s + Nfp * 2 * Np),
        u2s(u2r + Nfp * 2 * Np),
        udr(u2s + Nfp * 2 * Np),
        uds(udr + Nfp * 2 * Np),
        ubr(uds + Nfp * 2 * Np),
        ubs(ubr + Nfp * Np),
        dr(ubs + Nfp * Np),
        ds(dr + Np * Np),
        drsh(ds + Np * Np),
        lift(drsh + Np * 2 * Np),
        tau(lift + Np * 3 * Nfp),
        nr(tau + Nfp),
        ns(nr + Np),
        bf2n(ns + Np),
        w1(bf2n + Nfp * Nfp),
        w2(w1 + Nfp),
        tr1(w2 + Nfp),
        ts1(tr1 + Np * 2 * Np),
        tr2(ts1 + Np * 2 * Np),
        ts2(tr2 + Np * 2 * Np),
        g1(ts2 + Np * 2 * Np),
        g2(g1 + Nfp * Np),
        b2n(g2 + Nfp * Np),
        kv(b2n + Np * Np),
        total(kv + Nfp * 2 * Np) {}
};

// Edge kernel implementations (values as ARDG_EDGE_* in the C ABI).
// EDGE_AUTO picks EDGE_SPLIT where one thread per edge leaves the chip
// latency-bound (few waves per SIMD, or high order with few waves resident)
// and EDGE_LANE otherwise; split-BF16 products run on EDGE_SPLIT_MFMA up to
// N = 3 and on EDGE_MFMA above.
enum EdgeKernel { EDGE_AUTO = 0, EDGE_SPLIT = 1, EDGE_LANE = 2, EDGE_MFMA = 3, EDGE_SPLIT_MFMA = 4, EDGE_FIELDS = 5 };

// Diffusion coefficient forms (values as ARDG_D_* in the C ABI): one
// constant per field, or element-wise with the flux of Algorithm 1
// (reconstruction of D grad u~) or Algorithm 2 (reconstructed D times
// grad u~).
// DM_NODAL: a symmetric tensor (Dxx, Dxy, Dyy) at every node; DM_SOLUTION:
// the tensor D0 times the solution.  Both with Algorithm 1's nodal products.
enum DiffusionMode { DM_CONST = 0, DM_ALG1 = 1, DM_ALG2 = 2, DM_NODAL = 3, DM_SOLUTION = 4 };

// The compressible Navier-Stokes system in place of the scalar equation
// (values as ARDG_NS_* in the C ABI): off, Sutherland viscosity, or a
// constant viscosity.
enum NsMode { NS_OFF = 0, NS_SUTHERLAND = 1, NS_CONSTANT_MU = 2 };

struct DevMesh {
  int N = 0;
  int64_t K = 0, E_int = 0, E_bdy = 0;
  // interior edges: element index in bits 0..29, face in bits 30..31
  const int2* ef = nullptr;
  const double2* mu1 = nullptr;   // apex weights (lambda_w2, lambda_w3), side 1
  const double2* mu2 = nullptr;   // side 2
  const double2* gam = nullptr;   // gamma_R, gamma_S
  const int* bk = nullptr;        // boundary faces: element | face << 30
  const double2* bmu = nullptr;
  const double2* bgam = nullptr;
  const double2* vert = nullptr;  // [K][3] vertex coordinates
  const int* elem_face = nullptr; // [3][K] (edge << 1) | side
  const double* Delem = nullptr;  // [K] when D is element-wise
  const double2* vn = nullptr;    // [E] n1.v at A and at B (affine velocity)
  // prescribed exterior state at the nodes of each boundary face's ghost
  // sub-triangle (P2, B, A), [F][E_bdy][Np] at the current stage time, or
  // null (zero Dirichlet data through the mirror ghost)
  const double* ghost = nullptr;
  // tensor coefficient: nodal values [K][Np][3] (DM_NODAL) or D0 (DM_SOLUTION),
  // and per face (interior edges, then boundary faces) the parallelogram's
  // inverse metric (r_x, r_y, s_x, s_y) and sJ n1
  const double* Dnodal = nullptr;
  double D0[3] = {};
  const double4* gp = nullptr;
  const double2* sn = nullptr;
  const double* ops64 = nullptr;
  const float* ops32 = nullptr;
  int dmode = DM_CONST;           // DiffusionMode
  int edge_kernel = EDGE_AUTO;    // EdgeKernel
  int conv = 0;                   // convective term on
  int ns = NS_OFF;                // NsMode: the four fields are (rho, rho u, rho v, E)
  double gas[6] = {};             // gamma, R, Pr, mu_ref, T_ref, S (Sutherland constant)
  double Dfield[kMaxFields] = {};
  const double* Dfield_dev = nullptr;  // device copy of Dfield (read with scalar loads)
  double vel[6] = {};             // v = (p0 + p2 x + p3 y, p1 + p4 x + p5 y)
};

// What the element kernel does after forming du/dt for its element.
enum EpilogueKind { EPI_RHS = 0, EPI_RK4 = 1, EPI_LSERK = 2 };

struct Epilogue {
  int kind = EPI_RHS;
  int stage = 0;
  double dt = 0.0;
  double a = 0.0, b = 0.0;        // LSERK stage coefficients
  void* rhs_out = nullptr;        // EPI_RHS: [F][K][Np] in the compute type
  double* u = nullptr;            // FP64 state
  double* acc = nullptr;          // RK4 accumulator / LSERK residual (FP64)
  void* vnext = nullptr;          // next stage input in the compute type (may be null)
};

// One problem of a batch: its mesh tables and its buffers (one field).
struct BatchProb {
  DevMesh m;
  double* u = nullptr;      // FP64 state [K][Np] (caller-owned)
  double* acc = nullptr;    // RK accumulator (workspace)
  void* v = nullptr;        // stage vector in the compute type (workspace)
  void* flux = nullptr;     // edge fluxes in the compute type (workspace)
  double dt = 0.0;
};

// Edge fluxes of all interior and boundary edges for nfields fields.
hipError_t launch_edge_flux(const DevMesh& m, int prec, int nfields, const void* u, void* flux, hipStream_t st);
// Element volume + LIFT of the fluxes + epilogue (matrix cores).
hipError_t launch_element(const DevMesh& m, int prec, int nfields, const void* vin, const void* flux,
                          const Epilogue& epi, hipStream_t st);
// Batched (persistent) kernels over work items (problem, tile).  tile is the
// number of edges / elements per item and the block size (64, 128 or 256),
// or 0: side-split edge tiles (64 interior edges per item, items with a
// negative tile index are boundary tiles of 128 faces) and 64-element tiles
// on the matrix cores; grid is the number of persistent blocks.  in_u: the
// stage input is the FP64 state itself (FP64 stage 0 or LSERK); write_v: the
// element kernel writes the next stage input.
hipError_t launch_batch_edge(int N, bool fp64, int tile, int grid, const BatchProb* probs,
                             const int2* items, int nitems, int in_u, hipStream_t st);
hipError_t launch_batch_element(int N, bool fp64, int tile, int grid, const BatchProb* probs,
                                const int2* items, int nitems, const Epilogue& epi, int in_u,
                                int write_v, hipStream_t st);
// FP64 state -> FP32 stage vector for every problem of the items.
hipError_t launch_batch_to_f32(const BatchProb* probs, const int2* items, int nitems, int tile,
                               int Np, int grid, hipStream_t st);

// Edge kernel for a nodal tensor coefficient (DM_NODAL, DM_SOLUTION): one
// lane per face, FP64 and FP32 (same contract as launch_edge_flux).
hipError_t launch_edge_tensor(const DevMesh& m, int prec, int nfields, const void* u, void* flux, hipStream_t st);
// Navier-Stokes: interface fluxes sJ (F + G)* . n1 of the four conserved
// fields (Lax-Friedrichs + the aRDG viscous flux), [4][E][Nfp], and the
// element kernel (volume term, lift, epilogue) over all four fields.
hipError_t launch_edge_ns(const DevMesh& m, int prec, const void* q, void* flux, hipStream_t st);
hipError_t launch_element_ns(const DevMesh& m, int prec, const void* vin, const void* flux, const Epilogue& epi,
                             hipStream_t st);
// Edge kernel with interior edges on the matrix cores (same contract as
// launch_edge_flux).
hipError_t launch_edge_mfma(const DevMesh& m, int prec, int nfields, const void* u, void* flux,
                            hipStream_t st);
// Side-split tiles with the nodal -> Bernstein conversion on the matrix cores.
// Boundary faces with prescribed exterior data, one lane per face in a launch
// of their own (compute type FP64 or FP32), for the tiled launches (side-split
// and matrix-core): their tile kernels carry only the mirror-ghost boundary path, whose registers stay
// near the interior tiles' (the prescribed-state path holds about twice as
// many, and the allocation of a kernel covers every path in it).
hipError_t launch_boundary_faces(const DevMesh& m, bool f64, int nfields, const void* u, void* flux,
                                 hipStream_t st);
hipError_t launch_edge_split_mfma(const DevMesh& m, int prec, int nfields, const void* u, void* flux,
                                  hipStream_t st);
// Batched element kernel on the matrix cores (64-element tiles).
hipError_t launch_batch_element_mfma(int N, bool fp64, int grid, const BatchProb* probs, const int2* items,
                                     int nitems, const Epilogue& epi, int in_u, int write_v, hipStream_t st);
// Element kernel on the matrix cores (same contract as launch_element).
hipError_t launch_element_mfma(const DevMesh& m, int prec, int nfields, const void* vin, const void* flux,
                               const Epilogue& epi, hipStream_t st);
// Exterior state at the ghost nodes from its Chebyshev expansion in time on
// [ta, tb] (coeffs [n][nt], out [n]): at t = *tbase + toff when tbase is
// given (the stage time inside captured step graphs), else at t = toff.
hipError_t launch_ghost_eval(const double* coeffs, double* out, int64_t n, int nt, double ta, double tb,
                             const double* tbase, double toff, hipStream_t st);
// *t = value (one thread).
hipError_t launch_set_time(double* t, double value, hipStream_t st);
// *t += dt (one thread): the end of a step.
hipError_t launch_advance_time(double* t, double dt, hipStream_t st);
// Copy an FP64 state into an FP32 copy (stage input of the FP32 mode).
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);
// Count non-finite values of an FP64 array into *count_dev (int).
hipError_t launch_nonfinite(const double* x, int64_t n, int* count_dev, hipStream_t st);

}  // namespace ardg
