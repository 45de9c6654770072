"""FP64 CPU oracle of the fast-mode hot path (arXiv 2408.11472, Sec. III).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the HIP path is compared against.  Only the test
suite, the smoke check of the entry script and the CPU-baseline leg of the
benchmark may import it; the product path never does, and it shares no code,
tables or helpers with the HIP library.

Everything is float64 / complex128 NumPy.  numpy.fft serves as the FFT step
(a library primitive); every other step is written out as the paper (or, where
the paper is silent, the stated reading) defines it:

* ``surface``  - Choppy-Wave-Model fields and facets from the spectrum
                 (Sec. II.A, Sec. II.B "vertex, faces, normals");
* ``scatter``  - pulse-pair range, gate, Doppler bin, complex amplitude and
                 rasterisation into the Doppler-spectrum tensor (Sec. III.A,
                 Algorithm 1, Sec. II.A for the facet radar equation);
* ``iq``       - batched inverse DFT, eq. (1) weights and overlap-add into the
                 range-azimuth IQ matrix (Sec. III.B post-processing steps 1-4);
* ``fastmode`` - Algorithm 1 end to end;
* ``adjoint``  - multi-look waveform, L2 waveform loss and its gradient with
                 respect to facet heights and slopes (hand adjoint).

Parity status per function is stated in each module header.
"""

from . import surface, scatter, iq, fastmode, adjoint  # noqa: F401
