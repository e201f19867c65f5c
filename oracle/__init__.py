"""FP64 CPU oracle for ILS edge-preserving smoothing (Liu et al., "Real-time
Image Smoothing via Iterative Least Squares").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
The oracle shares no code with the GPU path: it takes plain NumPy arrays and
computes everything in float64 with NumPy / SciPy.

Modules
-------
ils      Algorithm 1 (Eqs. (1), (2), (7), (9), (11)) plus a dense direct
         solve of Eq. (8), the energy of Eq. (1) and the Welsch variant of
         Sec. 5 (Eqs. (19), (20)).
net      The learned-surrogate network (3x3 convolutions, ReLU, MSE, Adam) in
         float64 NumPy, forward and backward.  Not from the paper.

Parity status is recorded in each module's header.
"""
