"""CPU FP64 oracle for the Epstein-Nesbet MRPT2 energy (test infrastructure).

This package is test infrastructure only.  It is imported by the tests, by the
entry point's smoke check and by the benchmark's CPU-baseline leg, and by
nothing on the product path.  It shares no code with the HIP library: it
reads the same seeded synthetic inputs (package ``synth``) and computes the
same quantity from the paper's definitions:

  * primary space P = active strings in the allowed DAS categories, core
    fully occupied, virtuals empty (Sec. 2.4, STP-DAS categories);
  * external space Q = all single and double excitations out of P that are
    not in P (Sec. 2.3), optionally only those that touch core or virtual
    spinors;
  * Epstein-Nesbet partitioning: full H inside P, diagonal H_KK on Q
    (eq. zeroh);
  * E2 = sum_K |<K|H|Psi0>|^2 / (E0 - H_KK) (eq. pt2 / eq. pt2en), with
    Psi0 = C / ||C|| and E0 its Rayleigh quotient;
  * frozen core folded into h (h^FC in Sec. 2, notation list), frozen
    virtuals dropped (Sec. 2.5).

Modules:
  space      - DAS categories, reference strings, the external-space rule
  integrals  - two-electron integrals from Cholesky factors, frozen-core fold
  literal    - determinant-by-determinant E2 (Slater-Condon rules)
  classes    - the same sums organised by excitation class, vectorised over
               virtual spinors (for sizes the literal form cannot reach)
  counting   - closed-form external-space counts per class
  fullsize   - the class oracle on streamed factor columns, with the sums of
               the two-virtual classes as plain C loops (vvsum.c), for whole
               large workloads
"""
