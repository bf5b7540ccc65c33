"""Plain FP64 CPU oracle for the element-learning HDG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library.

Paper: "Element learning: a systematic approach of accelerating finite
element-type methods via machine learning, with applications to radiative
transfer" (arXiv 2308.02467).  Every function cites the section / equation it
follows.  The oracle computes what the paper defines in the most direct way:
dense assembly of the local matrices (eq. hdg_local_all_sub_mat), LAPACK LU
solves (eq. hdg_local_f2u_i2u), a sparse direct solve or a textbook GMRES for
the skeleton system (eq. hdg_global_mat), and recovery (eq. hdg_local_mat_sol).

Pins (what ties each function to something other than itself) live in
``tests/test_oracle_*.py``.  Functions without such a pin say
"parity unpinned" in their docstring.

Modules
-------
quadrature  LGL nodes, weights, differentiation matrix (Sec. 2.4.1)
angles      discrete ordinates and the phase matrix (Sec. 2.1, 2.2.1)
local       local HDG matrices and the in2out / in2sol / in2mean maps
            (Sec. 2.2.3, App. A)
mesh        skeleton numbering, element-to-trace maps, boundary data
            (Sec. 2.2.2)
trace       skeleton operator (I - P), direct solve and plain GMRES
            (eq. hdg_global_mat, Sec. 2.3)
recover     recovery, mean intensity, L2 error, energy balance
            (Alg. 1 step 4, eq. ang_ave)
dg          monolithic upwind DG for brute-force cross-checks (eq. dg)
mlp         FP64 fully connected network, MAE loss, Adam (Sec. 2.4.1, 3.1)
"""
