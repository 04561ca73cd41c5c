"""The C-ABI library: built, loadable without a GPU, exporting every entry
point include/nbody.h declares, and the Python binding declaring exactly
those entry points.  No compute calls (there may be no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("nbody_force", "nbody_predict", "nbody_correct", "nbody_blockstep",
                 "nbody_schedule", "nbody_energy", "nbody_create", "nbody_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_cs_0702135_amd._lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libnbody.so not built: run python -m paper_cs_0702135_amd.build")
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (nbody_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared()) <= exported


def test_binding_covers_exactly_the_header():
    import paper_cs_0702135_amd._lib as L
    assert sorted(L.SIGNATURES) == declared()
    lib = L.load()
    assert lib.nbody_version() >= 10000


def test_struct_layouts_match_header():
    import paper_cs_0702135_amd._lib as L
    # nbody_system: int64 n, 7 pointers, 5 doubles, uint32 flags (+ padding)
    assert ctypes.sizeof(L.NBodySystem) == 8 + 7 * 8 + 5 * 8 + 8
    assert ctypes.sizeof(L.NBodyForceConfig) == 7 * 4
    # nbody_ensemble_config: 2 int32, 6 doubles, 3 int32 (+ padding), 3 doubles
    assert ctypes.sizeof(L.NBodyEnsembleConfig) == 8 + 6 * 8 + 16 + 3 * 8


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_cs_0702135_amd._lib as L
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.nbody_create(ctypes.byref(h), 0, None) == L.NBODY_E_DEVICE
    assert lib.nbody_last_error(None) == b"null context"


C_PROGRAM = r"""
#include <stdio.h>
#include "nbody.h"

int main(void) {
    /* a host-only entry point: callable with no device */
    int64_t sizes[3] = {4096, 300, 1000};
    int32_t team_of[3], team_size[3], n_teams = 0;
    double secs[3];
    nbody_ensemble_config cfg = {3, 64, 30.0, 15.0, 0.5, 2.0e9, 247.0, 0.35, 4, 256, 2,
                                 6.0, 0.20, 0.81};
    int rc = nbody_ensemble_plan(sizes, 3, 96, &cfg, 0.0625, team_of, team_size, secs, &n_teams);
    if (rc != NBODY_OK || n_teams < 1 || n_teams > 3) return 1;
    if (team_size[team_of[0]] < team_size[team_of[1]]) return 2;
    rc = nbody_ensemble_plan(sizes, 0, 96, &cfg, 0.0625, team_of, team_size, secs, &n_teams);
    if (rc != NBODY_E_INVAL) return 3;
    printf("%d %d\n", nbody_version(), n_teams);
    return 0;
}
"""


def test_header_is_c_and_library_links_from_c(tmp_path):
    # the header compiles as C99 (no C++ in the boundary) and a C program
    # links against the library and calls it
    import paper_cs_0702135_amd._lib as L
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(L.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-L", libdir, "-lnbody", "-Wl,-rpath," + libdir, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    # the two small clusters share one single-group team, the large one has its own
    assert r.stdout.split()[1] == "2"
