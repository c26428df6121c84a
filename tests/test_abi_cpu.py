"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hodlr.h declares, orders points exactly as the
oracle's k-d ordering does, and rejects bad arguments before any device
work."""
import os
import re

import numpy as np
import pytest

import paper_1403_6015_amd as H
from oracle import hodlr_ref as hr
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hodlr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(?:hodlr_status|int32_t|void|const char\s*\*)\s*\**\s*(\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    L = H.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(H.EXPORTED) == names


@pytest.mark.parametrize("n,leaf", [(1, 1), (2048, 64), (1 << 20, 128), (1 << 22, 256), (1000, 7),
                                    (129, 128), (128, 128), (3, 1)])
def test_num_levels_matches_oracle(n, leaf):
    assert H.hodlr_num_levels(n, leaf) == hr.num_levels(n, leaf)


@pytest.mark.parametrize("dim,n,leaf", [(1, 1000, 16), (2, 777, 20), (3, 1500, 32), (2, 4096, 256),
                                        (2, 5, 1)])
def test_ordering_is_bit_exact_with_oracle(dim, n, leaf):
    rng = np.random.default_rng(dim * 1000 + n)
    x = rng.uniform(0, 1, (n, dim))
    # plant exact ties to exercise the tie rule
    x[n - 1] = x[0]
    if dim > 1:
        x[n - 2, 0] = x[1, 0]
    perm = H.hodlr_order(x, leaf)
    assert np.array_equal(perm, hr.kd_order(x, leaf))


def test_invalid_arguments_are_rejected():
    p = wl.se1d_small(64)
    bad = [
        dict(leaf=0),
        dict(tol=0.0),
        dict(tol=-1.0),
        dict(sigma2=-0.1),
        dict(theta=(0.0, 0.1)),
        dict(theta=(1.0, -0.1)),
        dict(kernel=7),
    ]
    for kw in bad:
        args = dict(x=p.x, y=p.y, kernel=p.kernel, theta=p.theta, sigma2=p.sigma2, leaf=p.leaf,
                    tol=p.tol)
        args.update(kw)
        with pytest.raises(H.HodlrError) as ei:
            H.gp_loglik(**args)
        assert ei.value.name == "EINVAL", kw
    xn = p.x.copy()
    xn[3, 0] = np.nan
    with pytest.raises(H.HodlrError) as ei:
        H.gp_loglik(xn, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    assert ei.value.name == "EINVAL"
    with pytest.raises(H.HodlrError) as ei:
        H.gp_loglik(np.zeros((4, 4)), np.zeros(4), p.kernel, p.theta, p.sigma2, p.leaf, p.tol)
    assert ei.value.name == "EINVAL"
    with pytest.raises(H.HodlrError) as ei:
        H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, H.Opts(max_rank=100000))
    assert ei.value.name == "EINVAL"
    # the sketch compressor's cap, and an unknown compressor
    for o in (H.Opts(max_rank=65, compressor=H.COMPRESS_SKETCH), H.Opts(compressor=2)):
        with pytest.raises(H.HodlrError) as ei:
            H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, o)
        assert ei.value.name == "EINVAL"


def test_per_point_noise_is_validated():
    """Per-point variances (§5's sigma_i^2): negative or non-finite values, a
    wrong length and the entry points that take none are rejected before any
    device work."""
    p = wl.se1d_small(64)
    for nz in (np.full(64, -0.1), np.r_[np.zeros(63), np.nan], np.r_[np.inf, np.zeros(63)]):
        with pytest.raises(H.HodlrError) as ei:
            H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, H.Opts(noise=nz))
        assert ei.value.name == "EINVAL"
        with pytest.raises(H.HodlrError) as ei:
            H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, H.Opts(noise=nz))
        assert ei.value.name == "EINVAL"
    with pytest.raises(ValueError):
        H.gp_loglik(p.x, p.y, p.kernel, p.theta, p.sigma2, p.leaf, p.tol,
                    H.Opts(noise=np.zeros(10)))
    with pytest.raises(H.HodlrError) as ei:
        H.Plan(64, 1, 16, H.Opts(noise=np.zeros(64)))
    assert ei.value.name == "EINVAL"



# C struct <-> ctypes mirror of the binding: sizes and every field's offset
_STRUCTS = [("hodlr_opts", "Opts"), ("hodlr_info_t", "Info"), ("hodlr_tune_t", "Tune"),
            ("hodlr_mlp_norm", "MlpNorm"), ("hodlr_sampler_cfg", "SamplerCfg"),
            ("hodlr_sampler_stats", "SamplerStats"), ("hodlr_profile_t", "Profile")]


def test_struct_layouts_match_the_header(tmp_path):
    """Compiles a C program against include/hodlr.h that prints sizeof and
    offsetof of every field the binding declares, and compares them with the
    ctypes structures (a mismatch would pass wrong options to the library)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hodlr.h"', "int main(void) {"]
    for cname, pname in _STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in getattr(H, pname)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, pname in _STRUCTS:
        cls = getattr(H, pname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
