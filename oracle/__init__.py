"""FP64 CPU oracle for recursive density-matrix perturbation theory in its
susceptibility form (Niklasson, Habib, Finkelstein, Rubensson, arXiv 2409.17033).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it. It shares no code with the HIP implementation.

Contents
--------
closed_form   D = theta(mu I - H) by eigendecomposition (Sec. II, the step
              function with Tr D = N_occ), chi^A and D^(1) by the
              Daleckii-Krein / Loewner formula (Appendix, proof of the
              Equivalence relation), expectation values and responses
              (Eq. expectation, Eq. direct, Eq. dual).
sp2           The SP2 recursion (Eq. DM0), its first-order response (Eq. DM1),
              the backward susceptibility sweep (Eq. DM2), the forward
              susceptibility sweep (Eq. DM3) and the merged forms
              (Eq. DMSuscept, Eq. DMPert), all in FP64 with full GEMMs.
finite_diff   Brute-force central differences of <A> = Tr[A D(H)] (definition
              of chi in Eq. Suscept) for tiny N.
scf           Self-consistent susceptibility (Eq. CP_SCF) and density response
              (Eq. DM_CP_SCF) for an on-site interaction, iterated with linear
              mixing as the paper writes them; the SCF ground state for FD.
mlp           The learned mixer network (forward, MSE loss gradient, Adam) in FP64.
nonorth       Non-orthonormal basis (Sec. V.A): congruences with an inverse
              factor Z, D = Z D_perp Z^T, chi_perp and the atomic-orbital
              chi_ao = Z chi_perp Z^T; the generalised-eigenproblem density.
fermi         Finite electronic temperature (Sec. V.B): the Fermi function with
              the canonical chemical potential, the temperature-dependent
              susceptibility with its mu_1 shift, and the recursive doubling
              expansion with its first-order response.

Pins (tests/test_oracle_*.py): hand-derived 2x2 closed forms, textbook
Rayleigh-Schroedinger first-order theory for diagonal H, brute-force finite
differences, exact-spectrum constructions, projector identities, the
commutator identity [H, chi] = [D, A], the duality identity for unconverged
recursions and the forward/backward equivalence.
"""
from . import closed_form, sp2, finite_diff, scf, mlp, nonorth, fermi  # noqa: F401
