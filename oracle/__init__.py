"""CPU FP64 oracle for the elastance and mobility integral equations (Rachh & Greengard,
"Integral equation methods for elastance and mobility problems in two dimensions").

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, links or calls this package;
only tests/, the smoke check in __graft_entry__ and the cpu_baseline leg of bench.py use it.
It shares no code with the HIP path: inputs come from the seeded generators in
paper_1507_05925_amd.workloads (curve samples and right-hand sides only), and every step of the
method is written out here again, plainly, in float64.

Contents
  nystrom   dense trapezoidal Nystrom assembly of (1/2 I + K + L) and (1/2 I + Kcal + L), right-hand
            sides, LU solve, outputs, elastance matrix P and mobility matrix M.
  matfree   the same operators applied matrix-free by plain C loops (for node counts where the
            dense matrix does not fit), GMRES via scipy, sampled-row applies.
  dirichlet the capacitance and resistance problems (the inverse problems of the paper's
            cross-tests) by completed double layers: dense operators, LU solves, the bounded
            solution with its charges / forces and torques and u_inf, the matrices C and R.

Parity status: every function is pinned by tests/test_oracle_*.py against closed forms, the
paper's tables, discrete Gauss-law identities, invariants or brute force; capacitance_field by
the exact two-disc exterior potential of the two-disc test (and the double layer's Gauss law).
The splash geometry is pinned through the paper's cross-tests with its printed potentials and
rigid motions; the nanocomposite geometry through the printed capacitances. Results that no pin
reaches: the splash potentials and velocities themselves (the paper prints only errors) and the
iteration counts (another discretization).
"""
