"""FP64 CPU oracle for the Hilbert-ordered spectral-element time step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code with the HIP library (no kernels, headers,
tables or helpers); the only shared module is ``workloads`` (seeded inputs).

What it computes (Araujo, Gross, Xavier-de-Souza, "Boosting Memory Access Locality of
the Spectral Element Method with Hilbert Space-Filling Curves", 2021):

* ``gll``      -- GLL nodes, weights and the nodal derivative matrix (Sec. 4.2,
                  Eqs. numerical_integ and deriv_u, on the tensor-product segment).
* ``mesh``     -- the local-to-global map mu(p, e), element geometry and the
                  element stiffness / lumped mass built from their definitions
                  (Sec. 4.2, Eqs. deriv_u, u_change, A-bar and R).
* ``reorder``  -- the Hilbert element reordering and the first-touch/degree node
                  reordering (Sec. 4.3, both enumerated procedures), plus the
                  Morton, lexicographic and seeded random element orders.
* ``solver``   -- explicit leapfrog stepping of the second-order acoustic system
                  with Ricker point sources and receivers (Sec. 4.2, Eq. u_change and
                  Alg. 3), the CFL time step and the discrete energy.
* ``adjoint``  -- the discrete adjoint of that recurrence and the gradient of an L2
                  receiver misfit with respect to per-element c^2.
* ``colour``   -- the greedy element colouring that makes the accumulation of Alg. 2
                  race-free (Sec. 5, the paragraph after Alg. 2).

Every floating-point quantity is FP64. Readings of passages where the paper is silent
or differs from this tensor-product, second-order setting are listed in the module
docstrings where they are used.
"""
