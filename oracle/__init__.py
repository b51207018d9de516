"""CPU reference (oracle) for the HDR-fused ptychography path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64 NumPy/SciPy code written from
the paper's equations and from the published reconstruction algorithms it
relies on.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the HIP library and
imports nothing from the product package.

Modules
-------
mnf      multi-scale non-linear fusion (Methods 3.4, Eqs. 5-10)
fourier  unitary 2D DFT (Eq. 3) and a brute-force DFT for tiny sizes
ptycho   exit wave (Eq. 2), Fourier-modulus projection, mini-batched
         ePIE / rPIE, Fourier error and NRMSE
adjoint  Poisson / amplitude loss on the far-field intensity and its
         gradient with respect to object and probe
unet     float64 reference of the warm-start network (forward, backward)
baselines linear-integration and single-exposure fusion, image metrics
broadband discrete-spectrum measurement (Eq. 4): resampling of a pattern per line
subpixel real-valued scan positions: Fourier-translated probe, mini-batched
         ePIE / rPIE at sub-pixel positions
mixed    mixed-state (multi-mode) probes: incoherent sum of modes, mini-batched
         ePIE / rPIE with a shared projection

Every function states the passage it follows; readings the paper leaves
open are named where they are used.
"""
