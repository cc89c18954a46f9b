"""The C-ABI library loads without a GPU and exports every entry point that
include/*.h declares; host-only entry points (validation, sizes,
compression-ratio arithmetic) run on the CPU."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for fn in os.listdir(INCLUDE):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(INCLUDE, fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:int|const char\*|void)\s+\**(csv_\w+)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    from paper_1311_1419_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1311_1419_amd import _native
    assert _declared() <= set(_native._SIGS)


def test_host_side_validation_and_sizes():
    import paper_1311_1419_amd as P
    p = P.Params(width=640, height=480, gop=16, block=32, m=256)
    assert p.resolve() == (256, 300)
    key, code, exp, bits = P.Context.encoded_size(p)
    assert (key, code, exp, bits) == (640 * 480, 15 * 300 * 256, 15 * 300, 15 * 300 * (8 * 256 + 8))
    assert P.Params(width=176, height=144, gop=4, block=32, m=0, rho=0.25).resolve() == (256, 30)
    for bad in (dict(block=8), dict(width=170), dict(gop=0), dict(m=1025), dict(iters=0),
                dict(key_qstep=24), dict(precision=7), dict(flags=256), dict(flags=512), dict(m=0, rho=0.0),
                dict(flags=P.CSV_FLAG_MEASURE_INT8 | P.CSV_FLAG_MEASURE_FP8),
                dict(flags=P.CSV_FLAG_WHOLE_FRAME | P.CSV_FLAG_MEASURE_FP8),
                dict(lambda_frac=float("nan"))):
        with pytest.raises(P.CsvError) as ei:
            p.with_(**bad).resolve()
        assert ei.value.code == -1
    for ok in (P.CSV_FLAG_MEASURE_INT8, P.CSV_FLAG_MEASURE_FP8,
               P.CSV_FLAG_MEASURE_FP8 | P.CSV_FLAG_ISTA, P.CSV_FLAG_TV):
        assert p.with_(flags=ok).resolve() == (256, 300)
    # whole frame: n = W H, one block per frame, M from rho over W H
    pw = p.with_(flags=P.CSV_FLAG_WHOLE_FRAME, m=0, rho=0.25)
    assert pw.resolve() == (76800, 1)
    assert P.Context.encoded_size(pw)[1:] == (15 * 76800, 15, 15 * (8 * 76800 + 8))
    with pytest.raises(P.CsvError) as ei:
        pw.with_(gop=33).resolve()
    assert ei.value.code == -2


def test_monotone_and_no_quant_flags():
    """MONOTONE selects the l1 solver (not with ISTA or TV); NO_QUANT keeps
    the exact int32 measurements (4 bytes and 32 bits per measurement, no
    exponent) and covers block DCT-l1 recovery only."""
    import paper_1311_1419_amd as P
    p = P.Params(width=640, height=480, gop=16, block=32, m=256)
    assert p.with_(flags=P.CSV_FLAG_MONOTONE).resolve() == (256, 300)
    for bad in (P.CSV_FLAG_MONOTONE | P.CSV_FLAG_ISTA, P.CSV_FLAG_MONOTONE | P.CSV_FLAG_TV):
        with pytest.raises(P.CsvError) as ei:
            p.with_(flags=bad).resolve()
        assert ei.value.code == -1
    for bad in (P.CSV_FLAG_NO_QUANT | P.CSV_FLAG_TV, P.CSV_FLAG_NO_QUANT | P.CSV_FLAG_WHOLE_FRAME):
        with pytest.raises(P.CsvError) as ei:
            p.with_(flags=bad).resolve()
        assert ei.value.code == -2
    nq = p.with_(flags=P.CSV_FLAG_NO_QUANT | P.CSV_FLAG_MONOTONE)
    assert P.Context.encoded_size(nq) == (640 * 480, 4 * 15 * 300 * 256, 15 * 300,
                                          15 * 300 * 32 * 256)


def test_compression_ratio_identity():
    import paper_1311_1419_amd as P
    p = P.Params(width=176, height=144, gop=5, block=16, m=64)
    cr = P.Context.compression_ratio(p, 40000, 4 * 99 * (8 * 64 + 8))
    assert cr["total"] == pytest.approx(5 / (1 / cr["key"] + 4 / cr["cs"]), rel=1e-12)
    raw = 8 * 176 * 144
    assert cr["key"] == pytest.approx(raw / 40000)
    assert math.isfinite(cr["total"])


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library the package refuses to run: loading it,
    and creating a decode context, raise instead of falling back."""
    import paper_1311_1419_amd as P
    from paper_1311_1419_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", os.path.join(ROOT, "no-such-dir", "libcsv.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(ImportError, match="HIP library not built"):
        _native.lib()
    with pytest.raises(ImportError, match="HIP library not built"):
        P.Context()
