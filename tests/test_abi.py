"""The C ABI library: loads without a GPU, exports every entry point that
include/hmc.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2002_01184_amd import hmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:hmc_status|const char\*|int32_t)\s+(hmc_\w+)\s*\(", src, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = hmc.lib()
    names = declared_symbols()
    assert {"hmc_init", "hmc_step", "hmc_sample_chain"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(hmc.EXPORTED) == names


def _target(kind=hmc.HMC_TGT_STD_NORMAL, dim=1, **kw):
    t = hmc.hmc_target(kind, 0, dim, None, None, hmc.HMC_F32, 0, 0, None, 1.0)
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _config(C=100, L=3, sd=hmc.HMC_F64, gd=hmc.HMC_F32, form=hmc.HMC_FORM_AUTO):
    return hmc.hmc_config(C, L, sd, gd, form, 0)


def test_workspace_size_and_validation():
    n1 = hmc.hmc_workspace_size(_target(), _config())
    n2 = hmc.hmc_workspace_size(_target(), _config(C=1000))
    assert 0 < n1 < n2
    bad = [(_target(dim=0), _config()), (_target(), _config(C=0)), (_target(), _config(L=0)),
           (_target(kind=9), _config()), (_target(kind=hmc.HMC_TGT_GAUSS_DIAG), _config()),
           (_target(kind=hmc.HMC_TGT_LOGREG, dim=3), _config(sd=hmc.HMC_F32))]
    for t, c in bad:
        with pytest.raises(hmc.HMCError) as e:
            hmc.hmc_workspace_size(t, c)
        assert e.value.status == hmc.HMC_E_INVALID
    # supported-combination checks
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_workspace_size(_target(), _config(sd=hmc.HMC_BF16))
    assert e.value.status == hmc.HMC_E_UNSUPPORTED
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_workspace_size(_target(), _config(sd=hmc.HMC_F32, gd=hmc.HMC_BF16))
    assert e.value.status == hmc.HMC_E_UNSUPPORTED


def test_init_rejects_bad_arguments_without_device_work():
    t, c = _target(), _config()
    n = hmc.hmc_workspace_size(t, c)
    fake = ctypes.c_void_p(4096)         # never dereferenced: validation fails first
    for steps, ws, nbytes, status in [([0.0], fake, n, hmc.HMC_E_INVALID), ([float("nan")], fake, n, hmc.HMC_E_INVALID),
                                      ([1.5, 1.5], fake, n, hmc.HMC_E_INVALID),
                                      ([1.5], ctypes.c_void_p(4100), n, hmc.HMC_E_INVALID),
                                      ([1.5], fake, n - 1, hmc.HMC_E_NOMEM)]:
        with pytest.raises(hmc.HMCError) as e:
            hmc.hmc_init(t, c, ctypes.c_void_p(8192), steps, ws, nbytes, None)
        assert e.value.status == status
    with pytest.raises(hmc.HMCError):
        hmc.hmc_init(t, c, None, [1.5], fake, n, None)
    assert hmc.lib().hmc_step(None, None) == hmc.HMC_E_INVALID
    assert b"ctx must not be NULL" in hmc.lib().hmc_last_error()
    assert hmc.lib().hmc_destroy(None) == hmc.HMC_OK


def test_workspace_sizes_across_targets_and_forms():
    # host-side carving for every target family, dtype pair and form the header admits; a
    # non-null pointer stands in for target data (workspace_size reads none of it)
    fake = ctypes.c_void_p(1 << 20)
    cases = []
    for form in (hmc.HMC_FORM_AUTO, hmc.HMC_FORM_PLAIN, hmc.HMC_FORM_FUSED, hmc.HMC_FORM_GRAPH):
        cases += [(_target(dim=1), _config(C=100, form=form)),
                  (_target(kind=hmc.HMC_TGT_GAUSS_DIAG, dim=1000, prec=fake), _config(C=16384, sd=hmc.HMC_F32, form=form)),
                  (_target(kind=hmc.HMC_TGT_GAUSS_DENSE, dim=100, prec=fake), _config(C=4096, sd=hmc.HMC_F32, form=form))]
        for D, N, xd in [(25, 1000, hmc.HMC_F32), (256, 100000, hmc.HMC_BF16), (512, 100000, hmc.HMC_BF16),
                         (300, 7000, hmc.HMC_F32)]:
            t = _target(kind=hmc.HMC_TGT_LOGREG, dim=D, X=fake, x_dtype=xd, n_rows=N, y=fake)
            for gd in (hmc.HMC_F32, hmc.HMC_BF16):
                cases.append((t, _config(C=8192, sd=hmc.HMC_F32, gd=gd, form=form)))
    sizes = []
    for t, c in cases:
        try:
            sizes.append(hmc.hmc_workspace_size(t, c))
        except hmc.HMCError as e:            # a combination the header lists as unsupported
            assert e.status == hmc.HMC_E_UNSUPPORTED, hmc.lib().hmc_last_error()
    assert len(sizes) >= len(cases) // 2 and all(s > 0 for s in sizes)


def test_noalloc_rejects_without_device_work():
    # the allocation-free entry point checks its size limit and form before any HIP call
    fake = ctypes.c_void_p(1 << 20)
    t = _target(kind=hmc.HMC_TGT_LOGREG, dim=256, X=fake, x_dtype=hmc.HMC_BF16, n_rows=100000, y=fake)
    c = _config(C=8192, sd=hmc.HMC_F32, gd=hmc.HMC_BF16)
    assert hmc.hmc_workspace_size(t, c) > hmc.HMC_NOALLOC_WORKSPACE_BYTES
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_sample_chain_noalloc(t, c, fake, [0.005], 10, 10, None, None, None, None, None, None)
    assert e.value.status == hmc.HMC_E_NOMEM and "exceeds" in str(e.value)
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_sample_chain_noalloc(_target(), _config(form=hmc.HMC_FORM_GRAPH), fake, [1.5], 10, 10, None, None,
                                     None, None, None, None)
    assert e.value.status == hmc.HMC_E_UNSUPPORTED
    with pytest.raises(hmc.HMCError) as e:
        hmc.hmc_sample_chain_noalloc(_target(), _config(), fake, [1.5], -1, 10, None, None, None, None, None, None)
    assert e.value.status == hmc.HMC_E_INVALID


def test_peak_helpers_reject_bad_arguments():
    st = hmc.lib().hmc_peak_compute
    out = ctypes.c_double(0.0)
    assert st(9, 8, 10, 1, None, ctypes.byref(out), None) == hmc.HMC_E_INVALID          # kind
    assert st(0, 0, 10, 1, None, ctypes.byref(out), None) == hmc.HMC_E_INVALID          # waves per SIMD
    assert st(0, 9, 10, 1, None, ctypes.byref(out), None) == hmc.HMC_E_INVALID
    assert st(0, 8, 0, 1, None, ctypes.byref(out), None) == hmc.HMC_E_INVALID           # iterations
    assert st(0, 8, 10, 1, None, None, None) == hmc.HMC_E_INVALID                        # output
    mem = hmc.lib().hmc_peak_memory
    assert mem(None, 1 << 20, 0, 1, 1, None, ctypes.byref(out)) == hmc.HMC_E_INVALID      # buffer
    assert mem(ctypes.c_void_p(16), 1 << 20, 2, 1, 1, None, ctypes.byref(out)) == hmc.HMC_E_INVALID   # mode
    assert mem(ctypes.c_void_p(8), 1 << 20, 0, 1, 1, None, ctypes.byref(out)) == hmc.HMC_E_INVALID    # alignment
    assert mem(ctypes.c_void_p(16), 1 << 20, 1, 2, 1, None, ctypes.byref(out)) == hmc.HMC_E_INVALID   # copy passes
    assert mem(ctypes.c_void_p(16), 8, 0, 1, 1, None, ctypes.byref(out)) == hmc.HMC_E_INVALID         # size
