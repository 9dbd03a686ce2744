"""Host logic of the launch-shape autotuner (no device): the choice rule, the
cache key and the JSON cache round trip."""
import json

from paper_2601_01437_amd import autotune
from paper_2601_01437_amd import binding as B


def test_pick_best_keeps_default_within_noise():
    assert autotune.pick_best([(0, 1.00), (128, 0.995), (512, 1.2)]) == (0, 1.00)
    assert autotune.pick_best([(0, 1.00), (128, 0.90), (512, 0.895)]) == (128, 0.90)
    assert autotune.pick_best([(0, 1.00), (128, 1.10), (512, 0.50)]) == (512, 0.50)


def test_shape_key_names_what_shapes_the_kernel():
    k1 = autotune.shape_key("gfx", B.IRL_TUNE_LUT_BLOCKS, 20, 10, 10, 1 << 20, 3, hidden=256)
    k2 = autotune.shape_key("gfx", B.IRL_TUNE_LUT_BLOCKS, 20, 10, 10, 1 << 20, 3, hidden=128)
    assert k1 != k2 and "H=256" in k1 and "lut_blocks" in k1
    p1 = autotune.shape_key("gfx", B.IRL_TUNE_PULL_BLOCKS, 20, 10, 10, 1 << 20, 3, hidden=256)
    p2 = autotune.shape_key("gfx", B.IRL_TUNE_PULL_BLOCKS, 20, 10, 10, 1 << 20, 3, hidden=128)
    assert p1 == p2 and "H=" not in p1
    assert autotune.shape_key("other", B.IRL_TUNE_PULL_BLOCKS, 20, 10, 10, 1 << 20, 3) != p1


def test_candidates_start_with_the_default():
    for name, kind, cands in autotune.KNOBS.values():
        assert cands[0] == 0 and len(set(cands)) == len(cands)
        assert kind in B.STAT_KINDS


def test_cache_round_trip(tmp_path):
    path = tmp_path / "sub" / "tune.json"
    c = autotune.TuneCache(str(path))
    assert c.get("k") is None
    c.put("k", 512, 0.25, [(0, 0.3), (512, 0.25)])
    c.save()
    data = json.load(open(path))
    assert data["k"]["value"] == 512 and data["k"]["timings"] == [[0, 0.3], [512, 0.25]]
    c2 = autotune.TuneCache(str(path))
    assert c2.get("k") == 512
    autotune.TuneCache(None).save()   # no path: nothing written


def test_binding_loads_torch_before_the_library():
    """The library must share torch's HIP runtime, so the binding imports torch
    before it loads the library (checked in a fresh interpreter)."""
    import subprocess
    import sys
    code = ("import sys, builtins\n"
            "order = []\n"
            "real = builtins.__import__\n"
            "def imp(name, *a, **k):\n"
            "    if name in ('torch', 'ctypes') and name not in order: order.append(name)\n"
            "    return real(name, *a, **k)\n"
            "builtins.__import__ = imp\n"
            "import ctypes\n"
            "real_cdll = ctypes.CDLL\n"
            "def cdll(path, *a, **k):\n"
            "    if 'libirlnqs' in str(path): order.append('lib:' + str('torch' in sys.modules))\n"
            "    return real_cdll(path, *a, **k)\n"
            "ctypes.CDLL = cdll\n"
            "import paper_2601_01437_amd.binding\n"
            "print([o for o in order if o.startswith('lib:')])\n")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "['lib:True']"
