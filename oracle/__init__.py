"""Plain CPU FP64 oracle for the FFT homogenization hot path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package; the product (the HIP library and its Python binding) never does.

The oracle shares no code with the GPU path. It is deliberately slow and
plain: numpy in float64, the discrete Fourier transform from ``numpy.fft``
(checked against a direct triple sum on tiny grids), Green operators written
as the tensor expressions they are, the constitutive laws of the paper's
Sec. 4 integrated by implicit Euler with a bisection for the one scalar
equation, and textbook fixed-point / conjugate-gradient / Newton iterations.

Modules
-------
tensor   Mandel notation, isotropic projectors.
fourier  direct DFT, FFT wrappers, discrete frequency vectors.
green    projector P(n) (Sec. 3.2, laminate equation), isotropic-reference
         Green operator, thermal operators.
laws     isotropic linear thermoelastic law and the PA66 law (Sec. 4).
solver   the periodic cell problem (Sec. 2, micro cell problem) on a voxel grid.

Every function carries "parity unpinned" in its docstring where no test pins
it to something other than itself.
"""
