"""CPU oracle for the periodic coupled-cluster Green's function (test infrastructure).

This package is a plain, slow, float64/complex128 restatement of what the GPU
path computes, used ONLY by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product path never imports it, and
it shares no code with the HIP library (only the seeded input generator).

Modules
-------
fock    O0: Fock-space brute force (Jordan-Wigner), straight from the operator
        definitions of the CC Green's function (Eqs. 4-8) with Lambda = T^dagger.
ktensor Momentum-blocked tensors and a k-conserving einsum (the bookkeeping of
        Eq. 9: every index carries a crystal momentum, blocks conserve it).
eom     O1/O2: similarity-transformed Hamiltonian blocks, EOM-IP/EA-CCSD sigma
        products, right-hand sides b and left vectors e, for any k-mesh
        (a single k-point is the molecular case).
unfold  O3: Bloch blocks -> Gamma-point supercell, for the k-point validation
        against a supercell calculation (Supporting Information, Sec. I).
solve   Dense inversion and the oracle's own restarted GMRES for the shifted
        systems of Eq. 6, and G = e . x of Eq. 7.
mor     O4: model-order-reduction frequency interpolation (MOR paragraph).
mlp     O5: reference forward/backward of the small network used for the
        learned initial guess.

Parity status of each function is stated in its module header.
"""
