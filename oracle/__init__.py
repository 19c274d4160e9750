"""Plain FP64 CPU oracle for the fourth-order cut-cell multigrid method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The HIP library never calls it and shares no code with it.

The oracle follows the paper step by step in the paper's notation:

* ``geometry``   -- cut cells and cell merging (Section 3, Algorithm 1)
* ``stencil``    -- ghost filling and the symmetric FV formulas (Section 4.1)
* ``discretize`` -- SFV/PLG classification, poised lattices, weighted
                    minimum-norm fits and the linear system (Sections 4.1-4.3)
* ``multigrid``  -- block smoother, transfers, V-cycle, outer iteration and
                    the two-grid operator (Section 5)
* ``rhs``        -- cell and boundary averages of given functions (eqs. (4.1)-(4.2))

Functions whose result is not pinned by a test against something the paper or
the mathematics fixes say "parity unpinned" in their docstring.
"""
