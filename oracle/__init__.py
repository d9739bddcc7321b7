"""Plain FP64 CPU oracle for first-order density-matrix perturbation theory.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls anything here; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do.  The oracle shares no
code with the HIP path: its only common dependency is the seeded input module
``workloads`` (random draws, no density-matrix arithmetic).

Modules
  exact      -- P0 = theta(mu I - H0) from the eigendecomposition (Eq. theta)
                and P1 from the Daleckii-Krein / sum-over-states closed form
                (Sec. IV, divided differences); invariants; finite differences
                (Eqs. FnD_2, FnD_4); Gershgorin bounds.
  control    -- the decisions of Algorithms 1-3 (sigma rule, D0 test,
                parameter-free D1 test) on FP64 scalars.
  sp2pt      -- Algorithms 1-3 run densely in FP64 (the layer recursion of
                Eq. S_n detailed with the bias of Eq. dB).
  eigsim     -- the same recursion run in the eigenbasis of H0, where each
                layer is a scalar map of eigenvalues and a Hadamard scaling of
                V^T S^(1) V (the block-function result of Mathias used in
                Sec. IV); gives exact per-layer matrices.
  constants  -- C_pt, the inflection points of the sigma-flip maps, and the
                contraction bound behind the 4.5 factor of the D0 test.
  adjoint    -- reference gradients of L = Tr(P1 W).

Parity status of each function is stated in its docstring.  Every part is
pinned; the 4.5 factor of the D0 test (Algorithm 2), which the paper takes
from earlier work, is pinned by the exact contraction bound of a sigma-flip
pair (constants.D0_PAIR_BOUND = 4.409 < 4.5).
"""
