"""The paper's transfer experiment (Table 1) as a probe: every strategy moves
the state correctly in both directions and both host memory kinds (the probe
checks the data it moved), and the per-amplitude strategy costs far more per
byte than one whole-state copy, as the paper reports."""

import pytest

from tests.gpu_util import ensure_built, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("to_device", [True, False])
def test_transfer_strategies_move_the_state(to_device, pinned):
    from paper_2309_16979_amd.msv import probe_transfer
    n = 16
    res = {}
    for strat in ("sync", "per_amplitude", "staged_remap"):
        log("transfer", strat, "h2d" if to_device else "d2h", "pinned" if pinned else "pageable")
        res[strat] = probe_transfer(n, strat, to_device, pinned, max_calls=1 << 12)
        assert res[strat]["seconds"] > 0
    assert res["per_amplitude"]["calls"] == 1 << 12 and res["staged_remap"]["calls"] == 2
    assert res["per_amplitude"]["seconds"] > 10 * res["sync"]["seconds"]
