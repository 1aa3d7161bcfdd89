"""CPU checks of the HIP library's boundary: it loads, exports every symbol the
header declares, and its host-only entry points (plan, peek) agree with the
oracle.  No compute call is made without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcbz.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2310_09467_amd import build, pcbz

    if not os.path.exists(pcbz.LIB_PATH):
        build.build()
    return pcbz.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcbz_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    from paper_2310_09467_amd import pcbz

    assert declared_functions() == sorted(pcbz.EXPORTS)


def declared_params():
    """{name: [parameter declarations]} from the header."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(pcbz_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text):
        args = " ".join(m.group(2).split())
        out[m.group(1)] = [] if args in ("", "void") else [a.strip() for a in args.split(",")]
    return out


def test_binding_argument_counts_match_header(lib):
    decl = declared_params()
    assert sorted(decl) == declared_functions()
    for name, params in decl.items():
        assert len(getattr(lib, name).argtypes) == len(params), name


def test_batch_call_takes_selector_arguments():
    """The batch call of the boundary takes the selector and its confidence
    threshold as arguments, after the per-frame inputs and before the outputs."""
    params = declared_params()["pcbz_compress_batch"]
    names = [re.findall(r"[A-Za-z_0-9]+$", p)[0] for p in params]
    assert names == ["ctx", "n", "prm", "d_frames", "d_prevs", "d_forced", "sel", "min_conf", "d_outs", "caps",
                     "lens", "stream"]
    assert params[6] == "const pcbz_selector *sel" and params[7] == "float min_conf"


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_plan_matches_oracle(lib, orc):
    from paper_2310_09467_amd import pcbz

    for h, w, p, lv in [(225, 225, 15, 1), (2040, 2040, 15, 9), (1020, 1020, 15, 9), (2040, 1020, 15, 9),
                        (45, 3345, 15, 1), (60, 84, 6, 2)]:
        nb, bound = pcbz.plan(h, w, p, lv, 0x7)
        assert nb == orc.plan(h, w, p, lv)[1]
        assert bound > 2 * h * w


@pytest.mark.parametrize("h,w,p,lv,mask", [(224, 225, 15, 9, 7), (225, 225, 15, 0, 7), (225, 225, 15, 9, 0),
                                           (225, 225, 15, 9, 1 << 16), (182, 182, 91, 9, 7)])
def test_plan_rejects(lib, h, w, p, lv, mask):
    from paper_2310_09467_amd import pcbz

    with pytest.raises(pcbz.PcbzError) as e:
        pcbz.plan(h, w, p, lv, mask)
    assert e.value.code == pcbz.EINVAL


def test_peek_reads_oracle_container(lib, orc):
    from paper_2310_09467_amd import pcbz, synth

    f = synth.config1_frame()
    blob, choice = orc.compress(f, pitch=15, level=1, cand_mask=0x3)
    info = pcbz.peek(blob)
    assert (info["h"], info["w"], info["pitch"], info["level"], info["n_bands"]) == (225, 225, 15, 1, 2)
    with pytest.raises(pcbz.PcbzError) as e:
        pcbz.peek(blob[:-3])
    assert e.value.code == pcbz.EDATA


def test_create_without_gpu_fails_cleanly(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.pcbz_create(ctypes.byref(h), 0, 0) != 0
