"""Plain, slow FP64 CPU oracle for the PEPS branch-and-bound hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything here: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP library;
the only module both sides use is the seeded input generator ``workloads``.

Modules
-------
energy    Eq. (1) and Eq. (2) energies, Boltzmann weights of the min-shifted
          tables (Sec. 2).
exact     brute-force enumeration (Z, ground energy, prefix marginals) and the
          exact row-transfer contraction for narrow lattices.
linalg    SplitMix64 counter generator and the truncated-SVD protocol used by
          the boundary-MPS compression.
bmps      boundary-MPS contraction of the Boltzmann PEPS, row by row (Sec. 2,
          Fig. 1(c)-(d)) with two-site variational compression.
search    branch-and-bound (beam) search over conditional marginals (Sec. 2,
          Fig. 1(d)-(e)).
mlp       reference forward/backward of the learned branch proposal.

Parity status of every function is stated in its module header.
"""
