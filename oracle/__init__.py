"""Plain FP64 CPU oracle of the modal-time-stepping DGSEM residual on mixed meshes.

TEST INFRASTRUCTURE ONLY.  This package is a slow, direct transcription of the
discretisation (paper Sec. 2: weak form Eq. (1), Duffy collapse, modal time stepping of
Algorithm 1, LSERK integration) and of the load-balancing arithmetic (Sec. 3: Hilbert
ordering, contiguous SFC segments, Listing 1 timer attribution).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the library and its
binding never do.  It shares no code, tables or constants with the GPU path.
"""
