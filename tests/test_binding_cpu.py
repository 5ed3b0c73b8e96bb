"""Host-side behaviour of the Python binding's plan cache (no GPU): plans are
keyed on the stream, and host threads sharing a stream share one plan whose
executes are serialised."""
import threading



class _FakeStream:
    def __init__(self, h):
        self.cuda_stream = h


def test_plan_cache_keys_on_stream(monkeypatch):
    import torch

    from paper_0811_2535_amd import binding

    made = []

    class FakePlan:
        def __init__(self, n, batch, dtype):
            made.append((n, batch, dtype))

        def destroy(self):
            pass

    monkeypatch.setattr(binding, "Plan", FakePlan)
    monkeypatch.setattr(binding, "_plans", {})
    monkeypatch.setattr(torch.cuda, "device", lambda d: _NullCtx())
    dev = torch.device("cuda", 0)
    s1, s2 = _FakeStream(0x1000), _FakeStream(0x2000)
    a = binding.cached_plan(1024, 2, torch.complex64, dev, s1)
    b = binding.cached_plan(1024, 2, torch.complex64, dev, s1)
    c = binding.cached_plan(1024, 2, torch.complex64, dev, s2)
    assert a is b and a is not c and len(made) == 2
    # another host thread on the same stream shares the plan (and its lock)
    got = []
    th = threading.Thread(target=lambda: got.append(binding.cached_plan(1024, 2, torch.complex64, dev, s1)))
    th.start()
    th.join()
    assert got[0] is a and isinstance(a.lock, type(threading.Lock()))


class _NullCtx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
