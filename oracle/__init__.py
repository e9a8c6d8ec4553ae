"""Plain FP64 CPU oracle for the flexibly enlarged CG method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the HIP implementation.

Modules
-------
ecg        flexibly SRE-CG2 (Algorithm 3 with Algorithm 1 as its no-switch
           case), truncation, column deflation, split preconditioning, CG.
brute      basis-free definitions of the search subspaces in high precision
           (mpmath), used to pin ``ecg`` on tiny inputs.
precond    block-Jacobi IC(0) and factorised G*G^T preconditioners.
learned    the learned preconditioner: features, MLP forward/backward, the
           A-norm loss and its gradient, Adam.
"""
