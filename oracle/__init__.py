"""Plain CPU FP64 oracle for compressive spectral clustering (Tremblay, Puy,
Gribonval, Vandergheynst, "Compressive Spectral Clustering", ICML 2016).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, calls or links this
package.  It may be used by the test suite, by the smoke check of the package
entry point and by the CPU-baseline leg of the benchmark, nothing else.  It
shares no code, header, table or helper with the GPU library; the only thing
both sides consume in common is the seeded graph data written by ``synth``.

Everything here is written for a reader holding the paper: each function
follows one step of Alg. 2 (or the definition it relies on) with numpy/scipy,
in float64, without blocking or fusion.  The modules are

* ``philox``      counter-based random numbers (Philox4x64-10, Salmon et al.
                  SC'11) and the Gaussian / uniform draws built from them;
* ``laplacian``   normalized Laplacian L = I - D^-1/2 W D^-1/2 (Sec. 2.1);
* ``jackson``     Jackson-damped Chebyshev approximation of the ideal
                  low-pass h_lambda_c of Eq. (1) (Sec. 4.3);
* ``cheb``        polynomial filtering by p products with L (Sec. 2.1, fast
                  graph filtering);
* ``eigencount``  eigencount estimate and dichotomy on lambda (Sec. 4.3);
* ``sampling``    uniform sampling without replacement, Eq. (4);
* ``kmeans``      k-means on the sampled features (Alg. 2 step 6);
* ``interp``      Tikhonov interpolation Eq. (5) by conjugate gradient and
                  the hard labels of Sec. 4.1;
* ``csc``         the whole of Alg. 2;
* ``metrics``     adjusted Rand index (Hubert & Arabie);
* ``mlp``         float64 reference of the lambda_k bracket network.

Stream identifiers of the random draws: COUNT=1 (eigencount signals),
FEAT=2 (feature signals), SAMPLE=3 (sampling keys), KMEANS=4 (k-means++ draws),
MLP=5 (network initialisation and minibatch order).
"""
