"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/sfft.h, its structs have the layout a C compiler gives
them, and invalid arguments are rejected on the host before any device call.
"""
import ctypes
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1606_07407_amd import sfft
    if not os.path.exists(sfft.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return sfft


def test_exports_every_header_symbol():
    sfft = _lib()
    names = sfft.header_symbols()
    assert {"sfft_plan_create", "sfft_recover", "sfft_plan_destroy", "sfft_last_error",
            "sfft_sample_lines", "sfft_dft"} <= set(names)
    L = sfft.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", sfft.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported
    assert sfft.sfft_version() >= 100


def test_struct_layout_matches_c(tmp_path):
    sfft = _lib()
    src = tmp_path / "lay.c"
    fields = {"sfft_params": [f[0] for f in sfft.sfft_params._fields_],
              "sfft_signal_batch": [f[0] for f in sfft.sfft_signal_batch._fields_],
              "sfft_outputs": [f[0] for f in sfft.sfft_outputs._fields_],
              "sfft_tune_entry": [f[0] for f in sfft.sfft_tune_entry._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sfft.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                         text=True).stdout.splitlines())
    for st, fs in fields.items():
        cls = getattr(sfft, st)
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fs:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


BAD = [
    (dict(d=3, d1=2), -1), (dict(d=0), -1), (dict(N=63), -1), (dict(N=0), -1),
    (dict(k_max=0), -1), (dict(c=1.0), -1), (dict(prime_rule=7), -1), (dict(p_min=-1), -1),
    (dict(ladder_K=0), -1), (dict(eta=0.0), -1), (dict(tau_noise=-1.0), -1),
    (dict(max_rounds=0), -1), (dict(max_rounds=1000), -1), (dict(precision=5), -1),
    (dict(robust=2), -1), (dict(classifier=3), -1),
    (dict(sched_nt=(8, 0, 0, 0)), -1),               # 8 column tiles below p = 640
    (dict(sched_nt=(5, 0, 0, 0)), -1), (dict(sched_nt=(0, 0, 9, 0)), -1),
    (dict(sched_nt=(0, 1, 0, 0)), -1), (dict(sched_fft=3), -1), (dict(sched_fft=-1), -1),
    (dict(sched_dft_batch=65), -1), (dict(sched_dft_batch=-1), -1),
    (dict(d=300, d1=1, precision=0), -2),            # d2 beyond 256
    (dict(d=100, d1=1), -2),                         # FP32: 2 (S+1) = 202 real rows > 128
    (dict(d=6, d1=6, N=1024), -2),                   # N^d1 = 2^60 > 2^40
    (dict(k_max=20000, c=5.0), -2),                  # primes beyond the DFT size
    (dict(k_max=3300, c=5.0), -2),                   # first round needs p >= 16500 > 16384
    (dict(k_max=1700, c=5.0, precision=0), -2),      # FP64: p >= 8500 > 8192
    (dict(d=40, d1=1, ladder_K=4), -2),              # 2 (S+1) rows beyond 8 MFMA tiles
    # general partitions
    (dict(blocks=(2, 1)), -1),                       # sizes sum to 3, not d = 4
    (dict(blocks=(4, 0)), -1),                       # an empty block
    (dict(blocks=(1, 1, 1, 1), order=(0, 1, 1, 3)), -1),  # order repeats a coordinate
    (dict(order=(0, 1, 2, 4)), -1),                  # order leaves 0..d-1
    (dict(blocks=(1,) * 300, d=300, precision=0), -2),  # more than 256 blocks
    (dict(blocks=(5, 1), d=6, N=1024), -2),          # N^(largest block) = 2^50 > 2^40
    # 2D tilting
    (dict(d=2, N=64, tilt=1, d1=2), -1),             # tilting needs d1 = 1
    (dict(d=3, N=64, tilt=1), -1),                   # and d = 2
    (dict(d=2, N=64, tilt=1, tilt_abc=(3, 4, 5)), -1),      # b = 4 is not > 2N
    (dict(d=2, N=64, tilt=1, tilt_abc=(20, 129, 131)), -1), # not a triple
    (dict(d=2, N=64, tilt=1, tilt_abc=(34, 288, 290)), -1), # gcd(a, b) = 2
    (dict(d=2, N=64, tilt_abc=(17, 144, 145)), -1),  # a triple without tilt
    (dict(d=2, N=64, tilt=2), -1),
]


@pytest.mark.parametrize("over,status", BAD)
def test_plan_create_rejects(over, status):
    sfft = _lib()
    base = dict(d=4, N=1024, k_max=64)
    base.update(over)
    with pytest.raises(sfft.SfftError) as ei:
        sfft.sfft_plan_create(sfft.Params(**base), max_batch=1)
    assert ei.value.status == status
    assert len(sfft.sfft_last_error()) > 0


def test_session_null_arguments():
    sfft = _lib()
    L = sfft.lib()
    h = ctypes.c_void_p()
    p = ctypes.c_void_p(0)
    assert L.sfft_session_create(None, 1, p, None, ctypes.byref(h)) == sfft.SFFT_EINVAL
    assert L.sfft_session_create(None, 1, p, None, None) == sfft.SFFT_EINVAL
    assert L.sfft_session_request(None, p, p, None) == sfft.SFFT_EINVAL
    assert L.sfft_session_points(None, p, None) == sfft.SFFT_EINVAL
    assert L.sfft_session_feed(None, p, None) == sfft.SFFT_EINVAL
    assert L.sfft_session_finish(None, None, None) == sfft.SFFT_EINVAL
    assert L.sfft_session_destroy(None) == sfft.SFFT_OK


def test_null_arguments():
    sfft = _lib()
    L = sfft.lib()
    h = ctypes.c_void_p()
    assert L.sfft_plan_create(None, 1, ctypes.byref(h)) == sfft.SFFT_EINVAL
    p = sfft.Params(d=4, N=1024, k_max=8).to_c()
    assert L.sfft_plan_create(ctypes.byref(p), 0, ctypes.byref(h)) == sfft.SFFT_EINVAL
    assert L.sfft_plan_create(ctypes.byref(p), 1, None) == sfft.SFFT_EINVAL
    assert L.sfft_recover(None, None, None, None) == sfft.SFFT_EINVAL
    assert L.sfft_dft(None, None, 1, 7, None) == sfft.SFFT_EINVAL
    assert L.sfft_plan_destroy(None) == sfft.SFFT_OK
    assert L.sfft_plan_max_prime(None) == 0
    n = ctypes.c_int32(7)
    assert L.sfft_autotune(None, None, None, 0, 1, 3, None, 0, ctypes.byref(n), None) == \
        sfft.SFFT_EINVAL
    b = sfft.sfft_signal_batch()
    for args in [(None, 1, 1, 3), (None, 0, -1, 3), (None, 0, 1, 0)]:
        c_values, n_c, warmup, steps = args
        assert L.sfft_autotune(ctypes.byref(p), ctypes.byref(b), c_values, n_c, warmup, steps,
                               None, 0, ctypes.byref(n), None) == sfft.SFFT_EINVAL
    # a batch with NULL arrays is refused before any device call
    assert L.sfft_autotune(ctypes.byref(p), ctypes.byref(b), None, 0, 1, 3, None, 0,
                           ctypes.byref(n), None) == sfft.SFFT_EINVAL
    assert "autotune" in sfft.sfft_last_error()


def test_product_path_does_not_import_oracle():
    # the binding and library sources never reach the CPU oracle
    pkg = os.path.join(ROOT, "paper_1606_07407_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
