"""Reference oracle for the sparse-SYK OTOC hot path (García-García, Liu, Verbaarschot,
"Sparsity independent Lyapunov exponent in the SYK model").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product library (``paper_2311_00639_amd``) never imports, links or calls it, and
the two share no code: the oracle computes every quantity from the paper's plain
definitions (dense Majorana matrices, dense Hamiltonian, eigendecomposition,
explicit traces, per-qubit Pauli matrix elements), in float64 / complex128.

Modules
-------
splitmix   SplitMix64 stream and output function (the counter-based generator both
           sides implement from its published definition; Steele, Lea & Flood 2014).
ensemble   the sparse coupling ensemble of Eq. (1): K distinct 4-subsets and J draws.
pauli      Pauli strings as per-qubit labels; the Jordan-Wigner Majorana strings of
           supplement Eq. (S1); products by the single-qubit Pauli multiplication table.
dense      dense Majoranas, H, parity blocks, e^{zH} by eigh, the OTOC of Eq. (2) as an
           exact trace and as the random-state estimator of the supplement, the Green
           function of the supplement.
haar       counter-based Haar-random state over the full 2^(N/2) space.
matfree    per-row matrix elements of H for sampled rows at any N (no dense matrix).
commuting  closed forms for pairwise commuting terms: e^{zH} as a product of cosh/sinh
           factors and the random-state OTOC of a lone Majorana pair, on the full vector
           at any N it fits (Pauli strings applied one tensor axis at a time).
lyapunov   disorder averages, crossing times t* and the Eq. (5) / Eq. (6) fits of the
           finite-size-scaling analysis, written out with plain least squares.

One module is a CPU comparator rather than a definition: cpu_lanczos (with its C source
cpu_lanczos.c) is the plain matrix-free complex128 Lanczos that the benchmark times on the
host cores beside the GPU library.  It is checked against matfree's row products and is
never called by the library.

Functions with no pin against the paper or mathematics are marked "parity unpinned"
in their docstrings; at present there are none.
"""
