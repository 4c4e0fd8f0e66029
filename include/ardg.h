/*
 * ardg.h -- C ABI of the MI355X (gfx950) affine-reconstructed nodal DG library.
 *
 * The library evaluates the semi-discrete convection-diffusion right-hand side
 * on unstructured triangles (the paper's eq. convection_diffusion with s = 0),
 * in the fully reference form of eq.
 * NDG_diffusion_once_matrixForm_Fullyreference: per element the Dr/Ds volume
 * term with the element's affine factors and (J_f/J) LIFT_f of the face fluxes;
 * per interior edge the diffusive flux n . grad(u~) (or n . (D grad u~)~ for
 * element-wise D, Algorithm 1) sampled at the LGL nodes of the diagonal of the
 * enclosed parallelogram, u~ being the least-squares reconstruction of
 * Algorithm aRDG.  Time stepping: classic RK4, or the five-stage fourth-order
 * low-storage Runge-Kutta the paper integrates with.
 *
 * Conventions shared by every call:
 *  - Reference triangle I = {r,s >= -1, r+s <= 0}, vertices a1=(-1,-1),
 *    a2=(1,-1), a3=(-1,1); element map of eq. mapping_tri with the element's
 *    CCW vertices (v1, v2, v3).  Faces f1=(v1,v2), f2=(v2,v3), f3=(v3,v1).
 *  - Nodes: warp-and-blend nodes (blend parameter 0) whose edge nodes are the
 *    LGL points.  Order: lattice rows of increasing s, each row in increasing
 *    r (ardg_ops_export(ARDG_OPS_NODES)).  Np = (N+1)(N+2)/2, Nfp = N+1.
 *  - State layout: [F][K][Np] contiguous, node fastest, F fields.
 *  - Edge flux layout: [F][E][Nfp] with E = E_int + E_bdy; interior edges
 *    first, ordered by their side-1 element (the lower element index) and
 *    its face, then boundary faces ordered by element and face.  Values are
 *    given in side 1's counter-clockwise face order (A -> B) with side 1's
 *    outward normal; side 2 sees the negated values in reverse order.
 *  - Boundary faces: zero Dirichlet data through a mirror ghost element (the
 *    element reflected across the face carrying -u at mirrored points), or,
 *    after ardg_mesh_set_boundary_data, a prescribed exterior state on the
 *    ghost's half of the reconstruction parallelogram; the paper specifies no
 *    boundary treatment.
 *  - Device pointers are caller-owned device memory on the mesh's device.
 *    Host pointers are only read during the call (the library copies them).
 *  - Every call returns an ardg_status; 0 is success, negative values are
 *    errors, and ardg_last_error() gives a thread-local message.  No call
 *    aborts the process or throws across the ABI.
 *  - Handles are not thread-safe; distinct handles may be used concurrently.
 */
#ifndef ARDG_H
#define ARDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ardg_status;

enum {
  ARDG_OK = 0,
  ARDG_E_INVALID_ARG = -1,
  ARDG_E_MESH_ORIENTATION = -2,      /* an element with J <= 0 (not CCW) */
  ARDG_E_MESH_TOPOLOGY = -3,         /* non-manifold or inconsistently oriented edge */
  ARDG_E_DEGENERATE_PARALLELOGRAM = -4,
  ARDG_E_RECON_RANK = -5,            /* reconstruction system not of full column rank */
  ARDG_E_UNSUPPORTED = -6,           /* order or precision not built */
  ARDG_E_HIP = -7,                   /* a HIP runtime call failed */
  ARDG_E_OOM = -8,
  ARDG_E_NONFINITE = -9              /* non-finite value found by ardg_check */
};

enum { ARDG_FP64 = 0, ARDG_FP32 = 1, ARDG_BF16X3 = 2 };
enum { ARDG_RK4 = 0, ARDG_LSERK54 = 1 };
enum { ARDG_D_CONST = 0, ARDG_D_ELEMENT = 1, ARDG_D_ELEMENT_ALG2 = 2, ARDG_D_NODAL = 3, ARDG_D_SOLUTION = 4 };
enum { ARDG_VEL_NONE = 0, ARDG_VEL_AFFINE = 1 };
/* The compressible Navier-Stokes system (ardg_mesh_set_navier_stokes). */
enum { ARDG_NS_OFF = 0, ARDG_NS_SUTHERLAND = 1, ARDG_NS_CONSTANT_MU = 2 };
/* Edge kernel implementations (ardg_mesh_set_kernels). */
enum {
  ARDG_EDGE_AUTO = 0,        /* chosen per launch (default)                                 */
  ARDG_EDGE_SPLIT = 1,       /* two waves per 64-edge tile, one per side, vector unit        */
  ARDG_EDGE_LANE = 2,        /* one lane per edge, vector unit                               */
  ARDG_EDGE_MFMA = 3,        /* one wave per 64 edges on the matrix cores                    */
  ARDG_EDGE_SPLIT_MFMA = 4,  /* side-split tiles, nodal -> Bernstein on the matrix cores     */
  ARDG_EDGE_FIELDS = 5       /* one lane per edge for every field (constant D), the next field
                                loaded during the current one's flux                         */
};

/* ardg_ops_export selectors (row-major double arrays). */
enum {
  ARDG_OPS_NODES = 0,        /* [Np][2] reference coordinates (r, s)                      */
  ARDG_OPS_V = 1,            /* [Np][Np] Vandermonde of the library's orthonormal basis   */
  ARDG_OPS_DR = 2,           /* [Np][Np] d/dr on nodal values                              */
  ARDG_OPS_DS = 3,           /* [Np][Np] d/ds                                              */
  ARDG_OPS_MASS = 4,         /* [Np][Np] reference mass matrix                             */
  ARDG_OPS_LIFT = 5,         /* [Np][3*Nfp] reference LIFT (1D mass on [-1,1] per face)    */
  ARDG_OPS_FACE_NODES = 6,   /* [3][Nfp] node index of each face node, CCW                 */
  ARDG_OPS_ROT_PERM = 7,     /* [3][Np] (Pi_f u)_i = u[perm[f][i]]: face f -> hypotenuse   */
  ARDG_OPS_RECON_A = 8,      /* [2Np][Mp] least-squares system (library basis)             */
  ARDG_OPS_RECON_R = 9,      /* [Mp][2Np] its pseudo-inverse                               */
  ARDG_OPS_RECON_GRAD = 10,  /* [2Nfp][2Np] nodal data on the two sub-triangles (each in its
                                own frame) -> (d/dR, d/dS) of u~ at the diagonal nodes     */
  ARDG_OPS_ALG1_GRAD = 11,   /* [4Nfp][2Np] Algorithm 1 blocks U1R, U1S, U2R, U2S on the same
                                nodal sub-triangle data (flux = D1 (gR U1R + gS U1S)
                                - D2 (gR U2R + gS U2S))                                    */
  ARDG_OPS_N2B = 12,         /* [Np][Np] nodal values -> Bernstein coefficients on I       */
  ARDG_OPS_ALG2_W = 13,      /* [2][Nfp] Algorithm 2: reconstruction at the diagonal nodes of
                                a coefficient equal to 1 on side 1 / side 2 and 0 on the
                                other (D~ = D1 w1 + D2 w2 for element-wise constant D)      */
  ARDG_OPS_RECON_VALUE = 14  /* [Nfp][2Np] nodal data on the two sub-triangles (each in its
                                own frame) -> u~ at the diagonal nodes                      */
};

/* ardg_mesh_export selectors. */
enum {
  ARDG_MESH_EDGES = 0,       /* int32 [E_int][4]: e1, f1, e2, f2 (faces 0..2)             */
  ARDG_MESH_BFACES = 1,      /* int32 [E_bdy][2]: element, face                            */
  ARDG_MESH_EDGE_GEOM = 2,   /* double [E_int][8]: P1x, P1y, mu1_A, mu1_B, mu2_B, mu2_A,
                                gamma_R, gamma_S                                            */
  ARDG_MESH_BFACE_GEOM = 3,  /* double [E_bdy][6]: P1x, P1y, mu_A, mu_B, gamma_R, gamma_S  */
  ARDG_MESH_ELEM_FACES = 4,  /* int32 [K][3]: (edge index << 1) | side (0: side 1)         */
  ARDG_MESH_BFACE_GHOST_NODES = 5  /* double [E_bdy][Np][2]: physical points of the nodes of each
                                boundary face's ghost sub-triangle (P2, B, A) (the reference
                                nodes mapped with those vertices): where the exterior state
                                of ardg_mesh_set_boundary_data is sampled                    */
};

typedef struct ardg_ops_s* ardg_ops;
typedef struct ardg_mesh_s* ardg_mesh;
typedef struct ardg_batch_s* ardg_batch;

typedef struct {
  int64_t K, Np, Nfp, E_int, E_bdy;
  int32_t N, device;
  double min_J;                /* smallest element Jacobian                              */
  double min_area_ratio;       /* smallest parallelogram area / quadrilateral area       */
} ardg_mesh_info_t;

/* Reference operators of order N (sections "Nodal discontinuous Galerkin
 * method" and "Reconstruction"): nodes, orthonormal basis, Dr, Ds, M, LIFT, the
 * three node orderings, the (N+1)^2-unknown least-squares reconstruction and
 * the constant per-edge operators that follow from the parallelogram map being
 * affine (Algorithm aRDG).  Built in FP64 on the host.
 * N: 1..6.  node_family: 0 (warp-and-blend, blend parameter 0).
 * Errors: E_INVALID_ARG (null out), E_UNSUPPORTED (N or family), E_RECON_RANK. */
ardg_status ardg_ops_create(int32_t N, int32_t node_family, ardg_ops* out);

/* Copy one reference operator (selector ARDG_OPS_*) into dst[cap] as doubles.
 * n_written receives the element count (also when cap is too small, in which
 * case E_INVALID_ARG is returned and nothing is written). */
ardg_status ardg_ops_export(ardg_ops ops, int32_t which, double* dst, int64_t cap,
                            int64_t* n_written);
void ardg_ops_destroy(ardg_ops ops);

/* Build a mesh: connectivity, element geometry (eqs. mapping_tri_diff,
 * triangle_jacobian_a/b), the enclosed parallelogram of every interior edge
 * (section "Enclosed parallelogram": the maximum-area parallelogram whose
 * diagonal is the shared edge), the apex coordinates in each element's rotated
 * frame (section "Reordering nodes in the reference domain") and the two
 * constant factors gamma = n1 . (r'_x, r'_y), n1 . (s'_x, s'_y) of the
 * parallelogram; boundary faces get the mirror-ghost rhombus.
 * vxy: host [Nv][2] doubles; etov: host [K][3] int32, counter-clockwise.
 * face_bc: reserved, must be NULL (all boundary faces are zero Dirichlet).
 * device: HIP device ordinal, or -1 for a host-only mesh (setup and export
 * only; kernels refuse it).  Errors: E_INVALID_ARG, E_MESH_ORIENTATION,
 * E_MESH_TOPOLOGY, E_DEGENERATE_PARALLELOGRAM, E_HIP, E_OOM. */
ardg_status ardg_mesh_create(ardg_ops ops, const double* vxy, int64_t Nv, const int32_t* etov,
                             int64_t K, const int32_t* face_bc, int32_t device, ardg_mesh* out);
ardg_status ardg_mesh_info(ardg_mesh mesh, ardg_mesh_info_t* out);
/* Export a mesh table (selector ARDG_MESH_*); dst is host memory of cap bytes. */
ardg_status ardg_mesh_export(ardg_mesh mesh, int32_t which, void* dst, int64_t cap,
                             int64_t* n_written);
void ardg_mesh_destroy(ardg_mesh mesh);

/* Diffusion coefficient (eq. diffusion; element-wise form of eq.
 * NDG_diffusion_once_matrixForm_reference_general with Algorithm 1).
 * mode ARDG_D_CONST: D[nfields] host doubles, one constant per field.
 * mode ARDG_D_ELEMENT: D[K] host doubles (nfields must be 1); the flux is then
 * Algorithm 1's reconstruction of D grad u~.
 * mode ARDG_D_ELEMENT_ALG2: D[K] as for ARDG_D_ELEMENT, with the flux of the
 * alternative form (eq. NDG_diffusion_once_matrixForm_reference_general_
 * alternative, Algorithm nonconstDiff2): the reconstructed coefficient
 * D~ = RDG(D^1, D^2) at the diagonal nodes times n . grad u~; at boundary
 * faces the mirror ghost carries the element's own D.
 * mode ARDG_D_NODAL: a symmetric tensor coefficient, space-varying and
 * anisotropic (eq. NDG_diffusion_once_matrixForm_reference_general; the
 * shear equation's cross term is its off-diagonal): D[K][Np][3] host
 * doubles, (Dxx, Dxy, Dyy) at every node; Algorithm 1 with nodal products
 * (each element's D evaluated at its sub-triangle's nodes, D grad u~ formed
 * node by node, reconstructed again); a mirror ghost carries D at mirrored
 * points.
 * mode ARDG_D_SOLUTION: D[3] = (D0xx, D0xy, D0yy), the coefficient u D0 of
 * eqs. advection_diffusion_nonlinear and diffusion_shear (nonlinear: each
 * stage uses its own state), Algorithm 1 as for ARDG_D_NODAL; a ghost
 * carries D0 times its state.
 * Tensor modes: nfields 1, FP64 and FP32 only (E_UNSUPPORTED for BF16X3),
 * one edge kernel (ardg_mesh_set_kernels does not apply); every tensor must
 * be symmetric positive definite.
 * Scalar values must be finite > 0. */
ardg_status ardg_mesh_set_diffusion(ardg_mesh mesh, int32_t mode, int32_t nfields,
                                    const double* D);

/* Edge kernel implementation for this mesh's launches (ARDG_EDGE_*).  All
 * compute the same flux up to rounding (Algorithm aRDG, Algorithm 1); the
 * default ARDG_EDGE_AUTO takes the side-split tiles where one lane per edge
 * would leave the chip latency-bound (fewer than ~8 waves per SIMD, or
 * N >= 5; in FP64 from N = 5 on with the conversion on the matrix cores)
 * and one lane per edge otherwise (in FP32 with several constant-D fields,
 * ARDG_EDGE_FIELDS), and for ARDG_BF16X3 the matrix-core kernels
 * (side-split up to N = 3).  Split-BF16 products exist
 * only on the matrix cores, so with ARDG_BF16X3 the vector-unit choices
 * (ARDG_EDGE_SPLIT, ARDG_EDGE_LANE) run ARDG_EDGE_MFMA.  Drops the mesh's
 * captured step graphs.  Errors: E_INVALID_ARG. */
ardg_status ardg_mesh_set_kernels(ardg_mesh mesh, int32_t edge_kernel);

/* Prescribed exterior state at the boundary faces (inhomogeneous, time-
 * dependent Dirichlet data), replacing the zero-Dirichlet mirror ghost: the
 * ghost sub-triangle (P2, B, A) of each boundary face carries the state g at
 * its nodes (ARDG_MESH_BFACE_GHOST_NODES), so the reconstruction is
 * u~ = RDG(u1, g); the upwind convective flux takes u+ = g on the face.
 * coeffs: host [nfields][E_bdy][Np][nt] doubles, the Chebyshev coefficients
 * of g at each ghost node in tau = (2t - t_a - t_b) / (t_b - t_a) on
 * [t_a, t_b] (copied).  Every evaluation (ardg_rhs_eval at its t, each stage
 * of ardg_rk_step at its stage time) must lie in [t_a, t_b]; calls outside it
 * fail with E_INVALID_ARG.  nt = 0 clears the data (back to zero Dirichlet).
 * With element-wise D the ghost carries the element's coefficient.  Meshes
 * with boundary data cannot join a batch.  Errors: E_INVALID_ARG, E_OOM. */
ardg_status ardg_mesh_set_boundary_data(ardg_mesh mesh, int32_t nfields, int32_t nt, double t_a, double t_b,
                                        const double* coeffs);

/* The compressible Navier-Stokes equations (subsection on the Navier-Stokes
 * equations: eq. aRDG_Navier_Stokes with the stress of eq. NS_viscosity, the
 * heat flux of eq. NS_heatflux, kappa = Cp mu / Pr) in place of the scalar
 * equation.  The state has four fields, (rho, rho u, rho v, E), [4][K][Np];
 * the gas is ideal: p = (gamma - 1)(E - rho |u|^2 / 2), T = p / (rho R),
 * Cp = gamma R / (gamma - 1).  The inviscid flux at a face is Lax-Friedrichs
 * (lambda = the larger |u . n| + c of the two traces); the viscous flux at a
 * face is G . n of the aRDG reconstructions of u, v and T on the enclosed
 * parallelogram (values and gradients at the diagonal nodes), with mu and
 * kappa from the reconstructed T.  Every boundary face takes its exterior
 * state from ardg_mesh_set_boundary_data (four fields, conserved variables):
 * at the ghost sub-triangle's nodes for the reconstruction and at the face
 * nodes as the outer Lax-Friedrichs state; computing without it fails with
 * E_INVALID_ARG.  law: ARDG_NS_SUTHERLAND (mu = mu_ref (T/T_ref)^(3/2)
 * (T_ref + S)/(T + S)), ARDG_NS_CONSTANT_MU (mu = mu_ref), or ARDG_NS_OFF
 * (back to the scalar equation).  params: host doubles {gamma, R, Pr, mu_ref,
 * T_ref, S} (gamma > 1, R, Pr, T_ref > 0, mu_ref, S >= 0).  While it is on,
 * the diffusion coefficient and the velocity are not used, nfields must be
 * 4, and the precision FP64 or FP32 (E_UNSUPPORTED otherwise); the state
 * must keep rho > 0 and p > 0.  The mesh cannot join a batch.  Drops the
 * mesh's captured step graphs.  Errors: E_INVALID_ARG, E_OOM. */
ardg_status ardg_mesh_set_navier_stokes(ardg_mesh mesh, int32_t law, const double* params);

/* Velocity of the convective term of eq. convection_diffusion, for every
 * field: ARDG_VEL_NONE, or ARDG_VEL_AFFINE with v(x,y) = (p0 + p2 x + p3 y,
 * p1 + p4 x + p5 y), params[6] on the host (v = (-y, x) is {0,0,0,-1,1,0}).
 * Nodal collocation of v u, strong form, upwind flux; u+ = 0 outside. */
ardg_status ardg_mesh_set_velocity(ardg_mesh mesh, int32_t kind, const double* params);

/* du/dt for nfields fields (one RHS evaluation = one Runge-Kutta stage).
 * precision ARDG_FP64: u_dev, rhs_dev are double [F][K][Np];
 * ARDG_FP32: float [F][K][Np] (operators and arithmetic in FP32, operators
 * built in FP64); ARDG_BF16X3: float [F][K][Np] as FP32, with the operator
 * products split into BF16 hi/lo parts on the matrix cores (hi hi + hi lo +
 * lo hi, FP32 accumulation).  Enqueued on hip_stream (hipStream_t, NULL = default);
 * uses a flux buffer owned by the mesh.  t: the time of the prescribed
 * boundary data (the only term that depends on time).  Errors:
 * E_INVALID_ARG, E_UNSUPPORTED, E_HIP. */
ardg_status ardg_rhs_eval(ardg_mesh mesh, int32_t precision, int32_t nfields, const void* u_dev,
                          void* rhs_dev, double t, void* hip_stream);

/* ardg_rhs_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, but the edge fluxes go to a library-owned
 * 64 MiB device array (one per GPU, held until the process ends) instead of
 * a buffer allocated on first use, and the call makes no allocation.  The
 * fluxes need nfields * (E_int + E_bdy) * Nfp * (8 in FP64, 4 otherwise)
 * bytes; larger requests fail with E_INVALID_ARG.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (different
 * streams or threads) race; calls on one stream are ordered.  Errors as
 * ardg_rhs_eval. */
ardg_status ardg_rhs_eval_noalloc(ardg_mesh mesh, int32_t precision, int32_t nfields, const void* u_dev,
                                  void* rhs_dev, double t, void* hip_stream);

/* Edge fluxes only (the interior and boundary loop of Algorithm aRDG with the
 * diagonal flux; Algorithms 1 and 2 for element-wise D; for the Navier-Stokes
 * system the numerical flux (F + G)* . n1 of the four conserved fields,
 * inviscid and viscous together): flux_dev [F][E][Nfp] in the
 * precision's type, D included, each edge's values multiplied by its surface
 * factor sJ = |edge| / 2 (the factor the surface integral of the weak form
 * applies, so that the element kernel needs no edge lengths).  Interior edges
 * first in ardg_mesh_export(EDGES) order, then boundary faces; values at the
 * edge's LGL nodes in element 1's counter-clockwise order, the sign of element
 * 1's outward normal; t is the time of the prescribed boundary data.  A
 * parity hook for the edge kernel. */
ardg_status ardg_edge_flux_eval(ardg_mesh mesh, int32_t precision, int32_t nfields,
                                const void* u_dev, void* flux_dev, double t, void* hip_stream);

/* Bytes of device workspace ardg_rk_step needs for (scheme, precision, nfields). */
ardg_status ardg_rk_workspace_bytes(ardg_mesh mesh, int32_t scheme, int32_t precision,
                                    int32_t nfields, int64_t* bytes);

/* Advance the FP64 state u_dev [F][K][Np] by nsteps steps of size dt with the
 * classic RK4 (4 stages) or the five-stage low-storage RK (paper's integrator).
 * The state update is FP64 in every precision; in ARDG_FP32 the operators act
 * on an FP32 copy of each stage's input.  work_dev: caller-owned device memory
 * of ardg_rk_workspace_bytes bytes, 256-byte aligned.  The step loop is
 * captured once per (scheme, precision, nfields, buffers, step count, dt)
 * into HIP graphs of at most 256 steps, replayed as often as nsteps needs
 * (plus one graph for the remainder).  t0: the time at the start, for the
 * prescribed boundary data (evaluated at each stage's time: RK4 0, dt/2,
 * dt/2, dt; the low-storage scheme's stage times).  Errors: E_INVALID_ARG,
 * E_UNSUPPORTED, E_HIP. */
ardg_status ardg_rk_step(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields,
                         double* u_dev, void* work_dev, double t0, double dt, int32_t nsteps,
                         void* hip_stream);

/* Capture and instantiate the graphs that ardg_rk_step replays for exactly
 * these arguments (nsteps >= 1) without running them, so that a caller can
 * keep the capture cost out of a latency-critical or timed region.  Nothing
 * is enqueued.  Errors as ardg_rk_step. */
ardg_status ardg_rk_prepare(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields,
                            double* u_dev, void* work_dev, double dt, int32_t nsteps);

/* Kernel timing hook (profiling): `reps` Runge-Kutta stages in the
 * configuration of ardg_rk_step are captured into graph A, and the same
 * stages' element kernels alone into graph B; each is replayed once untimed
 * and once between HIP events on hip_stream.  Returns the average duration in
 * milliseconds of the edge kernel, (A - B) / reps (out_ms[0]), and of the
 * element kernel with its fused update, B / reps (out_ms[1]).  Changes u_dev
 * and the workspace (graph B repeats stages), so the state is not a solution
 * afterwards; reps must be a multiple of the scheme's stage count.
 * Synchronises the stream.  Errors as ardg_rk_step. */
ardg_status ardg_stage_timing(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields,
                              double* u_dev, void* work_dev, double dt, int32_t reps,
                              void* hip_stream, float* out_ms);

/* Batching: many independent meshes of uneven size and order advanced
 * together.  Each mesh must live on the same device, carry one field with a
 * constant diffusion coefficient (ardg_mesh_set_diffusion with ARDG_D_CONST)
 * and no velocity; the meshes are referenced, not copied, and must outlive the
 * batch.  Work is split into tiles (edges or elements of one mesh); per order
 * N, persistent kernels walk the tiles of all meshes of that order, and a whole
 * ardg_batch_step is one HIP graph launch.  Tile sizes and persistent grid
 * sizes are chosen per (device, order, precision) by timing candidates on
 * first use; tune_cache names a text file where the choices are kept across
 * processes (NULL: no file).  Errors: E_INVALID_ARG, E_UNSUPPORTED (a mesh with
 * element-wise D or a velocity), E_HIP, E_OOM. */
ardg_status ardg_batch_create(const ardg_mesh* meshes, int32_t n, const char* tune_cache,
                              ardg_batch* out);
/* Device workspace for ardg_batch_step (per mesh: RK accumulator, stage vector,
 * edge fluxes), 256-byte aligned. */
ardg_status ardg_batch_workspace_bytes(ardg_batch batch, int32_t scheme, int32_t precision,
                                       int64_t* bytes);
/* Advance every mesh i by nsteps steps of size dt[i] (host array): u_devs[i]
 * is mesh i's FP64 state [K_i][Np_i] on the device (host array of n device
 * pointers).  Same schemes and precisions as ardg_rk_step; results equal the
 * per-mesh ardg_rk_step up to rounding.  E_UNSUPPORTED if a mesh no longer
 * meets ardg_batch_create's conditions (exterior data, a velocity or another
 * diffusion form set since), before anything is enqueued. */
ardg_status ardg_batch_step(ardg_batch batch, int32_t scheme, int32_t precision,
                            double* const* u_devs, void* work_dev, const double* dt,
                            int32_t nsteps, void* hip_stream);
/* The tile shapes in use for order N and a precision (tuning them first if
 * needed): edges per edge tile (64, 128, 256 with one thread per edge, or 0:
 * side-split tiles of 64 interior edges on two waves), elements per element
 * tile (64, 128, 256 with one thread per element, or 0: 64-element tiles on
 * the matrix cores), and persistent blocks per compute unit. */
ardg_status ardg_batch_tiles(ardg_batch batch, int32_t precision, int32_t N, int32_t* edge_tile,
                             int32_t* elem_tile, int32_t* grid);
void ardg_batch_destroy(ardg_batch batch);
/* ardg_check for a batch: synchronise the stream and scan every mesh's FP64
 * state u_devs[i] (host array of n device pointers, [K_i][Np_i]) for
 * non-finite values (E_NONFINITE if any).  Errors: E_INVALID_ARG, E_HIP. */
ardg_status ardg_batch_check(ardg_batch batch, double* const* u_devs, void* hip_stream);

/* Synchronise the stream and scan the FP64 state for non-finite values
 * (E_NONFINITE if any).  u_dev: double [F][K][Np]. */
ardg_status ardg_check(ardg_mesh mesh, int32_t nfields, const double* u_dev, void* hip_stream);

const char* ardg_status_string(ardg_status s);
const char* ardg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ARDG_H */
