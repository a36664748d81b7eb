"""The C-ABI library loads and exports every function its header declares (CPU only)."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(fb_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("fb_create", "fb_sweep", "fb_summaries", "fb_destroy", "fb_get_state",
                     "fb_set_state", "fb_trace", "fb_debug_counts", "fb_create_batch"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1606_06659_amd import fbmc
    lib = fbmc.load()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(fbmc.EXPORTS) == _declared()


def test_defaults_and_errors_without_device():
    from paper_1606_06659_amd import fbmc
    o = fbmc.fb_default_options()
    assert (o.chains, o.burnin, o.tune_start, o.max_steps, o.w0, o.shrink_cap) == (1, 1000, 100, 15, 1.0, 200)
    assert fbmc.load().fb_strerror(-4) == b"numeric failure in a draw"
    # invalid inputs are rejected before any device call
    import numpy as np
    y = np.zeros((10, 4), np.int32)
    X = np.ones((4, 2))
    h = np.zeros(4)
    with pytest.raises(fbmc.FbError) as e:
        fbmc.fb_create(y, X, h, options=fbmc.fb_default_options(max_steps=10))
    assert e.value.code == fbmc.FB_EINVAL
    with pytest.raises(fbmc.FbError):
        fbmc.fb_create(-np.ones((10, 4), np.int32), X, h)
    with pytest.raises(fbmc.FbError):
        fbmc.fb_create(y, np.ones((4, 5)), h)            # L > N
    with pytest.raises(fbmc.FbError):
        fbmc.fb_create(y, X, np.array([0, np.nan, 0, 0.0]))
    with pytest.raises(fbmc.FbError):
        fbmc.fb_create(y, X, h, priors=dict(a=-1.0))
    many_rows = np.arange(36, dtype=float).reshape(9, 4) / 7.0
    with pytest.raises(fbmc.FbError):
        fbmc.fb_create(np.zeros((3, 9), np.int32), many_rows, np.zeros(9))
    fbmc.fb_destroy(None)   # no-op


def test_new_entry_points_reject_a_null_context():
    """Launch choices, the three-level calls and the Laplace mode fail cleanly
    (FB_EINVAL) on a NULL context, before any device call."""
    import ctypes as C
    from paper_1606_06659_amd import fbmc
    lib = fbmc.load()
    assert lib.fb_set_beta_lanes(None, 2) == fbmc.FB_EINVAL
    assert lib.fb_get_beta_lanes(None) == 0
    assert lib.fb_set_hyper_split(None, 1) == fbmc.FB_EINVAL
    assert lib.fb_get_hyper_split(None) == 0
    assert lib.fb_set_shift_fusion(None, 1) == fbmc.FB_EINVAL
    assert lib.fb_set_top_level(None, None) == fbmc.FB_EINVAL
    assert lib.fb_set_top(None, 0, C.c_double(1.0), None) == fbmc.FB_EINVAL
    assert lib.fb_get_top(None, 0, None, None, None, None, None) == fbmc.FB_EINVAL
    assert lib.fb_set_beta_update(None, fbmc.FB_BETA_LAPLACE) == fbmc.FB_EINVAL


def test_allocator_callbacks_must_come_in_pairs():
    """fb_options.dev_alloc without dev_free (or the reverse) is rejected
    before any device call."""
    import numpy as np
    from paper_1606_06659_amd import fbmc
    y = np.ones((4, 2), np.int32)
    X = np.ones((2, 1))
    h = np.zeros(2)
    for which in ("dev_alloc", "dev_free"):
        opts = fbmc.fb_default_options()
        if which == "dev_alloc":
            opts.dev_alloc = fbmc.DEV_ALLOC_FN(lambda n, u: None)
        else:
            opts.dev_free = fbmc.DEV_FREE_FN(lambda p, u: None)
        with pytest.raises(fbmc.FbError) as ei:
            fbmc.fb_create(y, X, h, options=opts)
        assert ei.value.code == fbmc.FB_EINVAL and "dev_alloc" in str(ei.value)
