"""O6: dark/flat field correction and negative logarithm (oracle, test only).

The detector records raw = exp(-d) (flat - dark) + dark (Beer-Lambert law
with the dark field, beam off, and the flat field, beam on without the
sample; Section "Laminography reconstruction", the paragraph after the
line-integral model), so the line integrals are recovered as

    d = -log((raw - dark) / (flat - dark))

before any reconstruction.  The paper does not say what happens where the
ratio is not positive (raw <= dark, or a dead pixel with flat <= dark); the
reading here clamps the ratio from below at `min_ratio` > 0 and treats a
pixel with flat - dark <= 0 as ratio = min_ratio.  Computed in float64.
Pinned in tests/test_oracle_prologue.py: the exact round trip with the
recording model, the clamping cases, and the FBP of corrected counts.
"""
import numpy as np


def flat_dark_log(raw, dark, flat, min_ratio):
    raw = np.asarray(raw, dtype=np.float64)
    dark = np.asarray(dark, dtype=np.float64)
    flat = np.asarray(flat, dtype=np.float64)
    den = flat - dark
    safe = den > 0
    ratio = np.where(safe, (raw - dark) / np.where(safe, den, 1.0), min_ratio)
    return -np.log(np.maximum(ratio, min_ratio))
