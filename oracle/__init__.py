"""FP64 CPU oracle for radiative-transport flame volume reconstruction.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It is independent of
the HIP library: no shared code, headers or tables; the only common module is
the seeded input generator ``synth``.

The arithmetic lives in ``rte_oracle.c`` (plain C, double precision); this
module marshals numpy arrays into it with ctypes.

Parity status of each function (what pins it, see ``tests/test_oracle_pins.py``):
  ray_table            pinned (chord closed forms, symmetry, point projection)
  render               pinned (Beer-Lambert, sigma = 0 affine line integral,
                       fine-quadrature limit, 90-degree symmetry, point projection,
                       per-view in-scatter grids in a constant medium)
  inscatter            pinned (closed form for constant fields, also at every face node of an
                       unevenly rounded box; sigma = 0 limit)
  inscatter (phase_g)  pinned (g = 0 reduces to the isotropic grid, sigma = 0
                       closed form, forward/backward brightening, |g| -> 1 limit)
  backproject_adjoint  pinned (adjoint identity, dense-matrix transpose)
  backproject_paper    pinned (hand-computed single-ray worked case)
  reconstruct          pinned (dense least-squares recovery, SIRT monotone residual,
                       EM step = dense formula with likelihood ascent, fixed point
                       with the phase function)
  render_grad          pinned (central differences of render, adjoint identity)
  philox4x32_10        pinned (uniformity, word independence, avalanche)
  sample_gain          pinned (mean one, requested spread)
  flame_mask / hull    pinned (threshold definition, hull contains the flame and
                       shrinks as views are added)
  reconstruct_ext      pinned (reduces to reconstruct, masked and hull properties,
                       stop rule)
  planck / band / lut  pinned (Stefan-Boltzmann integral, Wien peak, LUT vs
                       direct integral within the interpolation bound)
  temperature_fit      pinned (fixed point at the true temperature, residual descent, one and
                       two iterations from another start against the EM step on a dense
                       matrix rebuilt at each iteration's temperature)
"""
from .oracle import *  # noqa: F401,F403
