"""CPU checks of the C ABI: the library loads, exports every entry point that
``include/ope.h`` declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ope.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:ope_status|const char\*)\s+(ope_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("ope_create", "ope_destroy", "ope_step", "ope_energy", "ope_residual", "ope_solve",
                 "ope_apply_h", "ope_source_solve", "ope_gram", "ope_small_solve", "ope_update",
                 "ope_set_inner", "ope_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2511_06788_amd import ope
    L = ope.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(ope.SIGNATURES)


def test_status_strings():
    from paper_2511_06788_amd import ope
    for s in range(8):
        assert ope.ope_status_string(s) and ope.ope_status_string(s) != "unknown status"
    assert ope.ope_status_string(99) == "unknown status"


@pytest.mark.parametrize("kw,expect", [
    (dict(dim=4), "OPE_EINVAL"),
    (dict(N=0), "OPE_EINVAL"),
    (dict(N=10 ** 6), "OPE_EINVAL"),
    (dict(h=(0.0, 0.1, 0.1)), "OPE_EINVAL"),
    (dict(m=(0, 4, 4)), "OPE_EINVAL"),
    (dict(kinetic=-1.0), "OPE_EINVAL"),
    (dict(precision=5), "OPE_EUNSUPPORTED"),
    (dict(N=513, m=(40, 40, 40)), "OPE_EUNSUPPORTED"),
])
def test_create_rejects_invalid_arguments(kw, expect):
    from paper_2511_06788_amd import ope
    args = dict(dim=3, m=(4, 4, 4), h=(0.2, 0.2, 0.2), N=4, kinetic=1.0, precision=0)
    args.update(kw)
    n = int(np.prod(args["m"][:args["dim"]])) if args["dim"] in (2, 3) else 8
    V = np.zeros(max(n, 1))
    with pytest.raises(ope.OpeError) as ei:
        ope.ope_create(args["dim"], args["m"], args["h"], V, args["N"], kinetic=args["kinetic"],
                       precision=args["precision"])
    assert ope.STATUS_NAMES[ei.value.status] == expect


def test_null_arguments_rejected():
    from paper_2511_06788_amd import ope
    L = ope.lib()
    assert L.ope_step(None, None, 1.0, None) == ope.OPE_EINVAL
    assert L.ope_apply_h(None, None, None) == ope.OPE_EINVAL
    assert L.ope_destroy(None) == ope.OPE_OK
    out = ctypes.c_void_p()
    assert L.ope_create(ctypes.byref(out), None, 4, 0, None) == ope.OPE_EINVAL
    assert out.value is None
