"""FP64 CPU oracle for the affine-reconstructed nodal DG (aRDG) diffusion RHS.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library under ``paper_1912_06221_amd``) never calls it and
shares no code, tables or helpers with it.

The oracle is written from the paper (Song & Srinivasan, "An efficient
reconstruction algorithm for diffusion on triangular grids using the nodal
discontinuous Galerkin method"), plain and slow, in float64:

* ``reference_element``  -- 1D LGL nodes, triangle nodes, orthonormal basis,
  Vandermonde, Dr/Ds, mass and LIFT (section "Nodal discontinuous Galerkin
  method").
* ``mesh``               -- affine element geometry (mapping equations for the
  triangle and its Jacobians) and face connectivity.
* ``ardg``               -- node reordering, the enclosed parallelogram, the
  projection Vandermonde, the least-squares reconstruction and the diffusive
  flux on the diagonal (section "Affine reconstructed algorithm", Algorithm
  aRDG), plus Algorithm 1 for element-wise diffusion coefficients.
* ``rhs``                -- the semi-discrete right-hand side in the fully
  reference form (weak form), the upwind convective term, classic RK4 and the
  five-stage low-storage RK, and the cell-normalised error norms.

Every function cites the passage it follows.  Readings of places where the
paper is silent are stated in the docstrings where they are used.
"""
