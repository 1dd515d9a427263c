"""FP64 CPU oracle for tree-level matrix-element reweighting.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the two meet only in the seeded inputs of ``synth``.

What it computes is the plain definition of the reweighting result (the
parameter-reweighting ratio w' = w |M'|^2 / |M|^2 of the paper's teaRex
section, with the normaliser's 1/0 -> 0 guard and the normalise-then-multiply
order the same section gives for the reweighting step):

  |M|^2(p; card) = A_P * sum_hel sum_colours | sum_diagrams M_d |^2

* e+e- -> mu+mu- and u u~ -> e+e- g: every Feynman diagram written out with
  explicit 4x4 Dirac matrices (``ee_mumu``, ``uu_eeg``).
* g g -> t t~ g g: colour decomposition into 24 orderings of the four gluon
  generators on the top line, colour-ordered partial amplitudes by
  Berends-Giele recursion, colour matrix by brute-force summation over
  Gell-Mann matrices (``qcd_bg``, ``colour``).  This is a different algorithm
  from the diagram-by-diagram device path.
* g g -> t t~ t t~ (pure QCD): colour-dressed Berends-Giele recursion with
  every external colour index left open and explicit Dirac matrices, the two
  assignments of antitops to tops added with the Fermi sign
  (``qcd_dressed``); again not diagram by diagram.

Parity is pinned (``tests/test_oracle_*.py``) by closed forms, invariants,
brute force and exact scaling laws; see each module for what pins it.
"""
