"""CPU oracle for the structured-operator and FISTA hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle is plain NumPy in FP64 (complex128 for operators, Python integers
for integer Hadamard). Every operator result is the dense matrix-vector product
of eq. (2) with the matrix built entry by entry from its definition; the fast
algorithms the GPU path uses (FFTs, Walsh-Hadamard butterflies, mode products)
reach exactly that result up to rounding, so the dense product is the reference.
The solver oracle runs the iteration itself, step by step, on the dense matrix.

Tiers (all independent of the GPU path):

* ``dense``      -- dense constructors and the dense product (eq. 2);
* ``fista``      -- soft thresholding, constant-step FISTA / ISTA, power
                    iteration, regularisation rule, objective;
* ``structured`` -- slower-than-GPU but dense-free evaluations used where the
                    dense matrix does not fit: row blocks of a Toeplitz matrix
                    generated on the fly, Kronecker products by mode products
                    with dense factors, and an FFT64 cross-check;
* ``grad``       -- gradients by CPU float64 autograd through dense unrolled
                    FISTA;
* ``omp``        -- orthogonal matching pursuit with FP64 least squares.

Parity status of every function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""

from . import dense, fista, grad, omp, structured  # noqa: F401
