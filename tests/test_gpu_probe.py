"""mc_probe on the GPU: every kind returns a finite, positive figure of the
right scale, and the arguments are checked."""
import math

import pytest

pytestmark = pytest.mark.gpu


def _mc():
    import paper_0812_2964_amd as mc

    return mc


@pytest.mark.parametrize("kind", list(range(12)))
def test_every_probe_kind_reports_a_figure(kind):
    mc = _mc()
    iters = {3: 256, 5: 512, 9: 200, 10: 200, 11: 200}.get(kind, 1024)
    fig, sec, work, cyc = mc.probe(kind, iters)
    assert math.isfinite(fig) and fig > 0 and sec > 0 and work > 0
    if kind <= 4:  # lane-instructions/s: below 256 CUs x 256 lanes x 3 GHz
        assert 1e11 < fig < 256 * 256 * 3e9
    elif kind == 5:  # bytes/s of LDS reads
        assert 1e12 < fig < 1e15
    else:  # cycles per read, instruction or four-site step
        assert cyc > 0 and 1.0 <= fig < 1e4
    if kind >= 9:
        assert work == iters * 8  # eight four-site steps per row of 32


def test_probe_rejects_bad_arguments():
    mc = _mc()
    for kind, iters in ((12, 10), (-1, 10), (0, 0), (0, (1 << 24) + 1)):
        with pytest.raises(mc.MCError):
            mc.probe(kind, iters)
