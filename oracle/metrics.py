"""Error measures of Sec. 4.1 (eq. 4.2).  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    """Relative L2 difference sqrt(sum (a-b)^2 / sum (a^2 + b^2)) of eq. 4.2.

    Used for the density error and for the coefficient arrays alike; 0 when
    both arrays vanish.
    """
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.sum(a * a + b * b)
    if den == 0.0:
        return 0.0
    return float(np.sqrt(np.sum((a - b) ** 2) / den))
