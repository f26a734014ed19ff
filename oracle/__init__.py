"""FP64 CPU oracle for the semi-Lagrangian lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1910_13918_amd``) never imports it and shares no code with it; the one
module both sides use is ``paper_1910_13918_amd.workloads``, which only draws
seeded initial fields and holds none of the method's arithmetic.

The oracle is a literal, slow transcription of Wilde, Kraemer, Reith, Foysi,
"Semi-Lagrangian lattice Boltzmann method for compressible flows"
(arXiv:1910.13918), Sec. II:

* ``velocity``     -- D1Q5 Gauss-Hermite abscissae and weights (Sec. II.B,
                      Table I), D2Q25 tensor product, scaled Hermite tensors
                      H^(0..4) written out index by index (Sec. II.A).
* ``equilibrium``  -- equilibrium Hermite coefficients a_eq^(0..4) (Sec. II.A,
                      eq. (10)) and the 4th-order equilibrium as a literal
                      full contraction over all 2^n index tuples (eq. (9) with
                      the discrete weights of Sec. II.B); g_eq (Sec. II.D).
* ``grid``         -- cells with Gauss-Lobatto-Chebyshev support points
                      (Sec. II.E), absolute node coordinates, product-formula
                      Lagrange basis, brute-force cell search, exact integrals
                      of the shape functions for the mass monitor.
* ``sllbm``        -- one time step: back-trace x - dt*xi_i, boundary
                      treatment, interpolation (eq. (17)), moments (eqs.
                      (3)-(5)), BGK relaxation (eq. (16)); initialisation,
                      moments, mass.
* ``sllbm3d``      -- the same step in three dimensions (D3Q125, the paper's
                      outlook): 3^n-tuple equilibrium contraction, tensor
                      product of three axes, isothermal BGK.
* ``riemann``      -- exact solution of the 1-D Riemann problem for the ideal
                      gas (reference for the Sod shock tube of Sec. III.C).
* ``adjoint``      -- complex-step derivatives of the oracle, used as the
                      exact reference gradient for the adjoint.

Everything runs in float64 (or complex128 for complex-step derivatives).
"""
