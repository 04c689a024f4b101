"""Plain FP64 CPU oracle for the tensor butterfly apply (arXiv 2411.03029).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
helpers with the GPU path: the only thing the two sides have in common is the
documented plan file format (``planio``), which each side reads and writes
with its own code, and the seeded input generators, which live in a module of
their own that holds none of the method's arithmetic.

Modules
-------
kernels    kernel entry functions K(x_i, y_j) (section 2, section 4)
dense      the plain definition u = K f and its adjoint: brute force, FFT
           (Fourier) and FFT convolution (Helmholtz)
idqr       column interpolative decomposition by Householder column-pivoted
           QR (section 2.1)
tucker     Tucker-type ID of a small full tensor (section 3.1)
butterfly  tensor butterfly construction (Algorithm 1) and contraction
           (Algorithm 2), plus the conjugate-transposed contraction
planio     writer for the documented plan file
"""
