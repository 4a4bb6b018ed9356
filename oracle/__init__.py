"""FP64 CPU oracle for the SBP-SAT anisotropic elastic wave operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
constants generators with the HIP library; both sides start from the
definitions in Almquist & Dunham, "Elastic wave propagation in anisotropic
solids using energy-stable finite differences with weakly enforced boundary and
interface conditions" (arXiv 2003.12811).

The oracle is plain NumPy / SciPy-sparse in float64.  It follows the paper's
definitions literally:

* ``sbp``       1-D norm H, first derivative D1, and the adapted fully compatible
                narrow second derivative D2^FC(b) built from its SBP form
                (Sec. 4, Sec. 4.1).
* ``material``  stiffness tensor layouts and the transformed stiffness
                c = F J C F, rho~ = J rho (Sec. 3.2.1).
* ``geometry``  discrete metric terms from D1 (Sec. 3.3), Nanson normals.
* ``elastic``   the discrete elastic operator (Sec. 4.6-4.7, Theorem 1) and the
                boundary and interface SATs in their physical form
                (Sec. 5.1 eq. sat_traction, Sec. 5.2 eq. dirichlet_ansatz,
                Sec. 6 eq. scheme_interface), assembled face by face.
* ``timestep``  classical RK4 on (u, u_t) and the Christoffel time step (Sec. 7).
* ``sources``   Ricker wavelet, moment-matching point source and receivers
                (Sec. 7.4; the discrete delta function is cited in Sec. 7.3-7.4).

Parity status of every function is recorded in its module docstring; all
functions are pinned by ``tests/test_oracle_*.py``.
"""
