"""Host logic of the dynamic loss scaler (CPU: the counter is set by hand)."""
import torch  # noqa: F401

from paper_2507_19141_amd.loss_scale import DynamicLossScaler


def test_skip_halves_and_growth_doubles():
    s = DynamicLossScaler(init_scale=1024.0, growth_interval=3, device="cpu")
    s.counter.fill_(2)
    assert s.update() is False and s.scale == 512.0 and s.skipped == 1
    assert int(s.counter.item()) == 0
    for _ in range(2):
        assert s.update() is True and s.scale == 512.0
    assert s.update() is True and s.scale == 1024.0
    s.counter.fill_(1)
    s.min_scale = 1024.0
    assert s.update() is False and s.scale == 1024.0


def test_state_roundtrip():
    s = DynamicLossScaler(init_scale=64.0, device="cpu")
    s.counter.fill_(1)
    s.update()
    t = DynamicLossScaler(device="cpu")
    t.load_state_dict(s.state_dict())
    assert t.scale == 32.0 and t.skipped == 1
