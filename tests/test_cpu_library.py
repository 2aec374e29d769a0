"""The C-ABI library builds, loads and exports every entry point of include/msb.h (no GPU)."""
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "msb.h").read_text()
    return sorted(set(re.findall(r"\b(msb_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_names():
    from paper_2506_09551_amd import _capi
    assert sorted(_capi.exported_symbols()) == declared_symbols()


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2506_09551_amd import _capi
    if not _capi.LIB_PATH.exists():
        pytest.skip("library not built")
    lib = ctypes.CDLL(str(_capi.LIB_PATH))
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_create_rejects_invalid_model_without_gpu():
    """Argument validation happens on the host before any device call."""
    from paper_2506_09551_amd import _capi
    if not _capi.LIB_PATH.exists():
        pytest.skip("library not built")
    with pytest.raises(_capi.MsbError) as e:
        _capi.msb_create(1, 1, 1, [], 4.0)
    assert e.value.status == _capi.MSB_EINVAL
    with pytest.raises(_capi.MsbError):
        _capi.msb_create(6, 7, 1, [(0, 1, 1.0)], 4.0)
    with pytest.raises(_capi.MsbError):
        _capi.msb_create(6, 3, 3, [(0, 6, 1.0)], 4.0)


def test_surrogate_fallback_rule_matches_oracle():
    """The fallback rule is host code: checked here against the oracle's rule."""
    import numpy as np
    from oracle import mlp as omlp
    msb = pytest.importorskip("paper_2506_09551_amd")
    try:
        msb.lib()
    except OSError:
        pytest.skip("library not built")
    assert msb.msb_mlp_num_params() == omlp.num_params()
    rng = np.random.default_rng(4)
    mean = rng.uniform(0, 1, (16, 40)).astype(np.float32)
    sd = rng.uniform(0, 0.06, (16, 40)).astype(np.float32)
    for frac in (0.02, 0.05, 0.1):
        assert np.array_equal(msb.msb_mlp_fallback(mean, sd, frac), omlp.fallback_rows(mean, sd, frac))


def test_bench_refuses_more_than_one_gpu():
    """`bench.py --gpus 2` prints one JSON line naming the limit and exits with
    status 2 before it touches a GPU."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=str(ROOT))
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


@pytest.mark.parametrize("name", ["msb_opts", "msb_shape", "msb_info", "msb_system"])
def test_struct_layout_matches_header(name):
    """The ctypes mirrors of the structs list the header's fields in order
    (ints, doubles, pointers to them and fixed arrays)."""
    from paper_2506_09551_amd import _capi
    text = (ROOT / "include" / "msb.h").read_text()
    end = text.index("} " + name + ";")
    body = text[text.rindex("typedef struct {", 0, end):end]
    fields = re.findall(r"^\s*(?:int|double)\s*\*?\s*(\w+)(?:\[[^\]]*\])?;", body, flags=re.M)
    assert len(fields) > 3
    assert [f[0] for f in getattr(_capi, name)._fields_] == fields


def test_fallback_calibration_flags_every_bad_row():
    """calibrate_fallback (host code of the learned form) returns a spread
    threshold under which every validation row whose error exceeds eps falls
    back through the library's fallback rule, and no threshold when no row
    is bad."""
    import numpy as np
    from paper_2506_09551_amd import surrogate as S
    msb = pytest.importorskip("paper_2506_09551_amd")
    try:
        msb.lib()
    except OSError:
        pytest.skip("library not built")
    rng = np.random.default_rng(8)
    ref = rng.uniform(0, 1, (6, 10, 30))
    mean = ref + rng.normal(0, 0.02, ref.shape)
    sd = np.abs(rng.normal(0, 0.02, ref.shape))
    mean[2, 4] += 0.3                       # two bad rows with a large spread somewhere
    sd[2, 4, 7] = 0.25
    mean[5, 1] -= 0.2
    sd[5, 1, 3] = 0.18
    eps = 0.1
    frac = S.calibrate_fallback(mean, sd, ref, eps)
    peak = ref.reshape(6, -1).max(axis=1)
    err = np.abs(mean - ref).max(axis=2) / peak[:, None]
    for p in range(6):
        mask = msb.msb_mlp_fallback(mean[p].astype(np.float32), sd[p].astype(np.float32), frac)
        assert np.all(mask[err[p] > eps])
    assert S.calibrate_fallback(ref, sd * 0, ref, eps) == 0.0
