"""Plain FP64 CPU oracle for the optimal-dimensionality spherical harmonic
transform of Khalid, Kennedy & McEwen, "An Optimal-Dimensionality Sampling
Scheme on the Sphere with Fast Spherical Harmonic Transforms" (IEEE TSP 2014).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product (``paper_1403_4661_amd``) never imports it, and the two
share no code: no kernels, no helpers, no tables, no constant generators.
Seeded input generation lives in ``tests/inputs.py`` and holds none of the
method's arithmetic.

Modules
-------
legendre  scalar and spin-weighted associated Legendre tables (Sec. III-F,
          Appendix A), upward three-term recursion with adaptive rescaling.
sampling  colatitude placements: the equiangular set (Eq. equiangular_set),
          the alternating vector (Eq. sampling_latitude) and the
          condition-number-minimising greedy placement (Sec. III-D).
sht       inverse SHT (Eq. f_inverse_SHT, Procedure 2), forward SHT
          (alias removal in the sample domain, descending |m|, from Eqs.
          gtof_inverse and signal_update), both adjoints, the dense
          sampled-harmonic matrix for tiny L, and error metrics
          (Eqs. exp1:errors, exp2:errors).

Functions whose parity is not pinned by an independent check say
"parity unpinned" in their docstring; at present every public function has
at least one pin in ``tests/test_oracle_*.py``.
"""

from . import legendre, sampling, sht  # noqa: F401
