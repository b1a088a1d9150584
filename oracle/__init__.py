"""FP64 CPU oracle for the LQ-over-2D-grid KKT solve (Zafar & Manchester).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link
or execute anything in this package; only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (``paper_2304_04980_amd``): the only common code is the seeded
input generator ``lqgrid_synth``, which holds none of the method's arithmetic.

Contents (each module cites the passage it follows):
  stack      -- the stacked matrices A~, B~, Q~, R~, omega~, r_delta and
                Delta = A~ Q~^-1 A~' + B~ R~^-1 B~'  (Sec. II-A, II-B)
  kkt        -- brute-force symmetric KKT solve by dense LDL' (Sec. II-B)
  riccati    -- the K = N = 1 special case by the textbook Riccati recursion
  splitting  -- explicit Psi~, Xi~, Phi~, Omega~ and the closed forms
                Upsilon_L (Lemma 1) and P_S^-1 (Theorem 2)   (Sec. IV)
  slab       -- the same operators applied one time slice at a time, for sizes
                where the full U x U matrices do not fit (Sec. II-B, IV-B)
  pcg        -- Algorithm 1 (PCGM) with a pluggable preconditioner, plain CG
  nbjm       -- Algorithm 2 (NBJM) with fixed S outer and L inner sweeps
  residual   -- primal recovery and the relative KKT residual

Every reading of a garbled or ambiguous passage is stated where it is used,
in the docstring of the function that relies on it.  Parity status: every function here is pinned by a
``-m "not gpu"`` test in tests/test_oracle_*.py; none is "parity unpinned".
"""
