"""FP64 CPU oracle for the nonlinear-elasticity hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the smoke entry point and
the benchmark's CPU-baseline leg may import or call it; the product path
(the C-ABI library and its Python binding) never does, and it shares no
code with them.  Inputs come from the `synthetic` generators only.

What it computes (paper sections cited per function):

* materials  -- strain energies Psi(F) and first Piola stresses P = dPsi/dF
                for the compressible neo-Hookean law (M1) and the paper's
                Cook law with an isochoric / volumetric split (M2) (Sec. 2,
                Sec. 4 "Cook test"), and the cardiac-like law M4
                (exponential isotropic and fibre terms, volumetric penalty,
                the active stress of Sec. 4 "Heartbeat test").
* fem        -- P1 tetrahedral geometry, internal forces, the residual
                r(u) = f_int(u) - f_ext (the quasi-static balance of Sec. 2
                written as the gradient of the potential of Sec. 3, eq.
                "minimization"), the potential itself, dead tractions, the
                follower endocardial pressure and elastic Robin springs of
                the heartbeat test, and
                the tangent stiffness assembled as a sparse matrix from
                complex-step derivatives of P.
* newton     -- exact Newton (eq. "newton" with a direct sparse solve), over
                load schedules and the heartbeat's time steps.
* solvers    -- plain GMRES (right preconditioned, modified Gram-Schmidt),
                CG, the Eisenstat-Walker forcing term, L-BFGS two-loop
                recursion and the dense BFGS inverse update of Sec. 3, and
                the NK / iNK / BFGS outer loops (Sec. 3, App. A options).
* mixed      -- the twist test's quadratic displacement / linear pressure
                form with the incompressible neo-Hookean law (M3), 4-point
                degree-2 rule, complex-step tangent (Sec. 4 "Twist test").
* linear     -- textbook small-strain linear elasticity (B-matrix / Voigt;
                linear and quadratic tetrahedra, the divergence block),
                independent of everything above, used as a pin.

Parity pins live in tests/test_oracle_*.py (closed forms, invariants,
finite differences, brute force, special cases).
"""
