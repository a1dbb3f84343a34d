"""FP64 CPU oracle for the MH3D reconstruction hot path.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU product path
(``paper_2503_13802_amd``) never imports, links or calls anything here, and this
package never imports the product package: the two share no code.  Seeded inputs
reach both sides as plain arrays.

Modules
-------
langevin  Langevin function derivatives L^(n)(u) (paper Sec. 2 definition of L,
          analytic structure of its poles in App. E, Prop. 2).
model     PSF bank, receive sensitivity, the forward operator A = P H B and its
          adjoint by direct summation (tier 1) and by numpy FFTs (tier 2), and the
          second-difference regulariser (Sec. 3.2 eq. portz, Sec. 4.1 eq. dN,
          Sec. 4.2 eq. Amodel/finalR, Sec. 4.3 Table tab:ops).
solver    Objective, power-iteration step size, accelerated projected gradient
          (FISTA) exactly in the paper's recurrence (Sec. 4.3), and closed-form
          special cases used as pins.
philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11), used for the
          power-iteration start vector so that both sides draw the same numbers.
mhad      The closed-form native image of App. D (eq. mhad2, eq. mhadM).
unet      The warm-start network (not in the paper): a 3D U-Net in FP64 with an
          optional BF16 storage model, its loss and its gradients.

Parity status: every function is pinned by tests under ``tests/test_oracle_*``
against closed forms, mpmath, finite differences, brute force or identities,
except where a docstring says "parity unpinned".
"""
