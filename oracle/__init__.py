"""CPU oracle for the butterfly FIO path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import, call, link or run anything in this package.
It shares no code with the HIP path in ``paper_0809_0719_amd``:

* ``direct``    -- the exact operator eq:dfio by direct O(N^4) summation, in C
                   (OpenMP, FP64) with an independent numpy twin;
* ``butterfly`` -- the FP64 step-by-step model of the Sec. 4 algorithm that
                   the HIP kernels must reproduce level by level.
"""
