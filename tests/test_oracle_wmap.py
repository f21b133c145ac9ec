"""Pin for the contour weight summand of Eq. (2), 1 - exp(-C^2 / sigma^2),
at points where it has a closed form."""
import math

import numpy as np


def test_wmap_closed_forms(orc):
    s = 0.25
    c = np.array([0.0, s, 2 * s, 1.0, 0.5 * s], np.float32)
    w = orc.wmap(c, sigma=s)
    assert w[0] == 0.0
    assert w[1] == np.float32(1.0 - 1.0 / math.e)
    assert w[2] == np.float32(1.0 - math.e ** -4)
    assert w[3] == np.float32(1.0 - math.e ** -16)
    assert w[4] == np.float32(1.0 - math.e ** -0.25)
    cc = np.linspace(0, 1, 1001, dtype=np.float32)
    ww = orc.wmap(cc, sigma=s)
    assert (np.diff(ww) >= 0).all() and ww.min() == 0.0 and ww.max() < 1.0
