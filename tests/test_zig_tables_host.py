"""The ziggurat tables the GPU library loads (csrc/zig_tables.inc, solved by
Newton iteration in csrc/gen_tables.py) against the oracle's
(oracle/zig_tables.h, solved by bisection in oracle/gen_zig_tables.py): the
same 256-strip geometry of Section 3.1 (ziggurat figure), so W, K, F, r and v
must agree bit for bit.  Both files are parsed as text; neither generator is
run and no code is shared."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GPU_TABLES = os.path.join(ROOT, "paper_2605_05099_amd", "csrc", "zig_tables.inc")
ORACLE_TABLES = os.path.join(ROOT, "oracle", "zig_tables.h")


def _number(tok):
    tok = tok.strip().rstrip("uUlL")
    if "p" in tok.lower() and tok.lower().startswith(("0x", "-0x")):
        return float.fromhex(tok)
    if re.fullmatch(r"-?\d+", tok):
        return int(tok)
    return float(tok)


def _arrays(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    out = {}
    for name, body in re.findall(r"\b([A-Z_]+)\[256\]\s*=\s*\{([^}]*)\}", text):
        out[name] = [_number(t) for t in body.split(",") if t.strip()]
    for name, val in re.findall(r"\b([A-Z_]+_[RV])\s*=\s*([^;]+);", text):
        out[name] = _number(val)
    return out


@pytest.mark.parametrize("dist,gpu,orc", [("normal", "RP_ZN", "OR_NORM"), ("exponential", "RP_ZE", "OR_EXP")])
def test_gpu_tables_equal_oracle_tables_bitwise(dist, gpu, orc):
    g, o = _arrays(GPU_TABLES), _arrays(ORACLE_TABLES)
    for part in ("W", "F"):
        a = np.array(g[f"{gpu}_{part}"], dtype=np.float64)
        b = np.array(o[f"{orc}_{part}"], dtype=np.float64)
        assert a.shape == b.shape == (256,)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (dist, part)
    assert g[f"{gpu}_K"] == o[f"{orc}_K"], (dist, "K")
    assert all(isinstance(k, int) and 0 <= k < 2**53 for k in g[f"{gpu}_K"])
    for part in ("R", "V"):
        assert np.float64(g[f"{gpu}_{part}"]).view(np.uint64) == np.float64(o[f"{orc}_{part}"]).view(np.uint64)
