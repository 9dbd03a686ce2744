"""CPU oracle for the linear-method (LM) operator and the IRL optimisation step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It is a plain, slow, FP64
implementation written from the paper's Methods sections and shares no code,
tables or constants with the HIP library.

Modules
-------
``space``        fixed-(N_alpha, N_beta) determinant space (Methods, "Wave Function
                 Ansatz" and the particle-number constraint of "Autoregressive
                 Modeling and Physical Constraints").
``hamiltonian``  second-quantised Hamiltonian on a determinant set via the
                 Slater-Condon rules (Methods, "Wave Function Ansatz", Hamiltonian
                 equation).
``nqs``          one-hidden-layer real network, amplitude and Jacobian, i.e. the
                 tangent basis {psi, d psi / d theta_i} (Methods, "From SR to a
                 Stable Eigenvalue Problem", linearised wavefunction).
``lm``           dense S~, H~, energy centring, H_eff, the standard Hermitian
                 eigenproblem and the update (same section; Eqs. rayleigh_quotient,
                 full_gevp, heff, standard_evp), plus the matrix-free operator
                 apply used as the reference for every GPU apply.

Parity status (each function states its pin in the tests):
* enumeration, Slater-Condon elements and signs, NQS Jacobian, energy,
  gradient, dense LM matrices, modes A and G: pinned (see tests/test_oracle_*).
* mode P step length: parity unpinned (the paper gives no formula for the
  step length of the p x p problem; only its direction is defined).
"""
