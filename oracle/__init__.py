"""CPU oracle of the batched SNAP + Langevin fine propagator (FP64, plain, slow).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything in this
package.  It imports nothing from the product package and the product package
imports nothing from it.

* ``defn``     -- definition tier (NumPy + exact rationals): CG, Wigner-D by the
                  polynomial action, Z, B and the Wirtinger adjoint, for tiny inputs.
* ``oracle``   -- ctypes front end of ``snap_oracle.c`` (plain C, FP64, no FMA).
* ``parareal`` -- classical and adaptive parareal drivers over the C propagators.
"""
