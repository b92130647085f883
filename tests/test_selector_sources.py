"""The committed timing tables and the models fitted to them describe the
current kernels: each table and the network's weights record the digest of
the sources that decide what the SpMV kernels cost (kernels, launch
parameters, formats, interface; comments and layout ignored), and it must
equal the digest of the sources in the tree (CPU only)."""
import json
import os

import numpy as np

from paper_1210_2536_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1210_2536_amd")
TABLES = ["train_0000_2500.npz", "train_2500_5000.npz", "heldout_0000_0500.npz"]


def test_tables_and_weights_match_the_current_kernel_sources():
    digest = B.timing_sources_digest()
    for t in TABLES:
        d = np.load(os.path.join(PKG, "data", t))
        assert "sources" in d.files, t
        assert str(d["sources"]) == digest, f"{t} was measured on other kernels: re-collect"
    with open(os.path.join(PKG, "weights", "selector_gfx950.json")) as fh:
        w = json.load(fh)
    assert w["meta"]["kernel_sources_sha256"] == digest, "weights fitted to other kernels"


def test_digest_ignores_comments_but_not_code():
    a = "int f(int x) { return x + 1; } // add one\n/* note */"
    b = "int f(int x)\n{\n    return x + 1;  /* the increment */\n}\n"
    c = "int f(int x) { return x + 2; }"
    assert B._strip_comments(a) == B._strip_comments(b) != B._strip_comments(c)
    assert B._strip_comments('const char *s = "a // b /* c */";') == \
        'const char *s = "a // b /* c */";'
