"""FP64 CPU oracle of the quasi-cylindrical arbitrary-order PSATD PIC cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the smoke check and the CPU-baseline leg of the
bench do.  The oracle shares no code with the HIP path: it is written from
the paper (Jalas et al., "Accurate modeling of plasma acceleration with
arbitrary order pseudo-spectral particle-in-cell methods") with NumPy/SciPy
primitives (FFT, Bessel functions, matrix inverse, bincount) as its steps.

Modules
  spectral   finite-order modified wavenumber, radial grids, discrete Hankel
             transform pair, spectral operators, current correction, PSATD
  particles  linear-shape deposit and gather with the on-axis parity rule,
             Boris push, lattice injection
  cycle      the PIC cycle (gather/push -> deposit -> transforms -> PSATD ->
             inverse transforms -> moving window) and its state
  diag       beam diagnostics (emittance, slice energy spread) and the
             paper's error metrics
  stencil    stencil reach and numerical-dispersion/Cherenkov curves
"""
