"""MI355X-native EPIC (E-field Parallel Imaging Correlator) imaging path.

The compute lives in ``libepic.so`` (hand-written HIP for gfx950, C ABI in
``include/epic.h``); this package is its thin Python binding.
"""
from ._lib import (  # noqa: F401
    BATCH_QUEUE, EPIC_BF16X2_MFMA, EPIC_F8E4M3_MFMA, EPIC_F16_MFMA, EPIC_F32, EPIC_FIXED16, EXPORTS,
    FIXED_DEFAULT, MAX_SAMPLES_4BIT, MAX_SAMPLES_8BIT, NORMALISE, XFORM_AUTO, XFORM_DFT_DIRECT,
    XFORM_DFT_SEPARABLE, XFORM_FFT,
    JONES, REMOVE_AUTOS, STOKES, SUB_BANDED, VOLT_8BIT, Accumulator, EpicError, Graph, Plan, accumulate,
    accumulate_frames, grid, image, load, readout, readout_noalloc,
)
