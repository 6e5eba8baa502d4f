"""The serving arena's allocator (host logic, CPU memory): first fit, 256-byte granules,
freed ranges merged with their free neighbours, and the request sizes it carves."""
import pytest

torch = pytest.importorskip("torch")

from paper_2301_12796_amd import serve  # noqa: E402
import synth  # noqa: E402


def test_first_fit_and_merge():
    a = serve.Arena(10 * 256, "cpu")
    x = a.alloc(300)            # two granules
    y = a.alloc(256)
    z = a.alloc(1)
    assert (x, y, z) == (0, 512, 768) and a.in_use == 4 * 256
    assert a.alloc(7 * 256) is None                     # 6 granules left
    a.release(y, 256)
    assert a.alloc(512) == 1024                         # the hole of one granule is too small
    a.release(x, 300)
    assert a.free[0] == (0, 768)                        # merged with the hole at 512
    a.release(z, 1)
    a.release(1024, 512)
    assert a.free == [(0, 10 * 256)] and a.in_use == 0  # everything merged back


def test_request_buffers_fit_exactly():
    sensors = synth.serving_sensors()
    for cam, _ in sensors:
        need = serve.request_bytes(cam)
        px = sum((cam.width >> l) * (cam.height >> l) for l in range(3))
        assert px * 53 <= need < px * 53 + 18 * 256
        a = serve.Arena(need, "cpu")
        assert a.alloc(need) == 0 and a.alloc(1) is None
    bufs = serve._buffers(sensors[0][0], 3)
    assert [(l, side, name) for l, side, name, _, _ in bufs[:6]] == [
        (0, "live", "depth"), (0, "live", "vertex"), (0, "live", "normal"),
        (0, "model", "vertex"), (0, "model", "normal"), (0, "model", "mask")]
