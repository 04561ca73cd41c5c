"""Teardown order of the Python binding's library contexts (CPU only).

Contexts are destroyed by an atexit hook registered when the first one is
created, so that nbody_destroy (a stream synchronisation and frees) runs
while torch and the HIP runtime are still alive, not from a finaliser during
interpreter shutdown.  These checks use a stand-in for the library handle.
"""
import paper_cs_0702135_amd as nb


class _FakeLib:
    def __init__(self):
        self.destroyed = []

    def nbody_destroy(self, h):
        self.destroyed.append(getattr(h, "value", h))
        return 0


def _ctx(lib, h):
    c = object.__new__(nb.Context)
    c.lib, c.h, c.device = lib, h, 0
    return c


def test_close_all_destroys_each_context_once(monkeypatch):
    lib = _FakeLib()
    c1, c2 = _ctx(lib, 11), _ctx(lib, 12)
    monkeypatch.setattr(nb, "_ctx", {0: c1, 1: c2})
    nb._close_all()
    assert sorted(lib.destroyed) == [11, 12]
    assert nb._ctx == {}
    # the finaliser of a closed context makes no further library call
    c1.__del__()
    c2.__del__()
    assert sorted(lib.destroyed) == [11, 12]


def test_first_context_registers_the_exit_hook_once(monkeypatch):
    import ctypes

    registered = []
    monkeypatch.setattr(nb.atexit, "register", lambda f: registered.append(f))
    monkeypatch.setattr(nb, "_atexit_registered", False)
    monkeypatch.setattr(nb, "_ctx", {})
    monkeypatch.setattr(nb.torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(nb.torch.cuda, "current_device", lambda: 0)
    lib = _FakeLib()

    def fake_create(out, device, stream):
        ctypes.cast(out, ctypes.POINTER(ctypes.c_void_p))[0] = 100 + device
        return 0

    lib.nbody_create = fake_create
    monkeypatch.setattr(nb.L, "load", lambda: lib)
    a = nb.context(0)
    b = nb.context(1)
    assert nb.context(0) is a
    assert registered == [nb._close_all]
    nb._close_all()
    assert sorted(lib.destroyed) == [100, 101]
    del a, b
