"""Plain FP64 CPU oracle for the subspace-accelerated sigma-transformed Poisson solves.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH. Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it. The GPU library never calls it,
and it shares no code with the GPU library: it assembles the operator as a sparse matrix,
runs textbook restarted GMRES and Householder-QR least squares, and re-derives every
coefficient from the paper on its own.

Modules, each following the passage it cites:

* ``fd``            finite-difference weights (Fornberg 1988) and 1-D difference matrices
* ``discretization`` grid, sigma-transform geometry (Sec. 2.1), the mixed-stage operator
                     with ghost-node Neumann rows (Sec. 3, discrete pressure and Neumann
                     equations) and the low-order still-water preconditioner operator
* ``operator3d``    the mixed-stage operator on a (chi, gamma, sigma) grid (Sec. 2.1 in three
                     dimensions, Sec. 3)
* ``precond``       fixed preconditioners: vertical line Jacobi and an x-semicoarsening
                     V-cycle (the still-water preconditioner role of Sec. 3)
* ``gmres``         left-preconditioned restarted GMRES (Saad & Schultz 1986, Sec. 3)
* ``subspace``      EWMA sketch (Alg. 4) and the least-squares initial guess (Alg. 2)
* ``rangefinder``   randomized range finder over a sliding window of solutions (Alg. 3)
* ``rng``           the counter-based Gaussian stream that draws the sketch vectors
* ``sequence``      the per-system driver: guess, solve, push the solution into the sketch
* ``closedloop``    LSERK45 stepping of velocity and surface whose pressure systems feed the
                     solver (Sec. 3, Alg. 1)
* ``ilu``           ILU(0) of the still-water operator (Sec. 3's preconditioner)

Parity status of each function is stated in its module header; a function without an
independent pin says "parity unpinned".
"""
