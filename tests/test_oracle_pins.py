"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_rejects_bad_arguments(orc):
    import numpy as np

    x = np.zeros(4, dtype=np.complex64)
    with pytest.raises(ValueError):
        orc.forward(x, [2], [], 2, np.zeros(3))          # even order
    with pytest.raises(ValueError):
        orc.forward(x, [1], [], 2, np.zeros(2))          # wrong K
    with pytest.raises(ValueError):
        orc.forward(x, [1], [], 3, np.zeros(4), hist=np.zeros(1))  # history length


def test_empty_input(orc):
    import numpy as np

    z = orc.forward(np.zeros(0, dtype=np.complex64), [1, 3], [1], 3, np.ones(10))
    assert z.size == 0
    gx, gc = orc.backward(np.zeros(0), [1, 3], [1], 3, np.ones(10), np.zeros(0))
    assert gx.size == 0 and np.all(gc == 0)
