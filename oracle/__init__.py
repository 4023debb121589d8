"""Plain FP64 CPU oracle for the FE-DMN hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it builds the paper's explicit operators (gradient operator A, weight
matrix W, dense Newton Hessian A^T W D A with a LAPACK Cholesky, Milton's
laminate formula with the projector P(n)) where the GPU path condenses the
laminate tree block by block.

Modules
-------
mandel     Mandel basis, projector P(n) (Sec. 3.1), symmetrisation N(n) (Sec. 3.2),
           isotropic stiffness 3K P1 + 2G P2 (Sec. 4.4).
tree       Perfect binary laminate tree: weight propagation and volume
           fractions (Sec. 2.1), paper ordering of laminates (Sec. 3.1/3.2),
           dense gradient operator A (Sec. 3.2).
linear     Linear DMN homogenisation: bottom-up Milton laminate formula
           (Sec. 3.1) and the dense form of the algorithmic tangent (Sec. 3.2).
j2         J2 elasto-plasticity with exponential-linear hardening (Sec. 4.1),
           implicit Euler radial return and consistent tangent.
gp         Online evaluation at one Gauss point: Newton on the jumps with the
           dense Hessian, backtracking, convergence test of Sec. 4.6,
           effective stress and algorithmic tangent (Sec. 3.2).
grad       Gradients of the linear map by complex-step differentiation.
orientation  Fibre-orientation interpolation of the normals (Sec. 2.3).
compression  Tree compression of zero-weight subtrees (Sec. 3.1) and the
           linear map of the compressed tree.
training   Offline-training objective (Sec. 3.1), AMSGrad with the modulated
           learning rate (Sec. 4.5) and the stiffness sampler (Sec. 4.4).

Readings of points the paper leaves open are stated in each function's
docstring.
"""
