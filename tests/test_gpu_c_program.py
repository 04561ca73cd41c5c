"""The C ABI used from C on the GPU: a C99 program (compiled here with gcc
against include/nbody.h, libnbody.so and the HIP runtime) allocates device
memory with hipMalloc, calls nbody_force (Section 2, Eq. (1)) on a seeded
Plummer sphere, then nbody_init and five nbody_blockstep steps, and writes the
results; the pair sums are compared with the float64 oracle (acceleration
p99 <= 1e-6, max <= 1e-5, float32 mode) and the block steps must have
advanced every particle's time consistently."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from tests.gpu_util import need_gpu, rel_vec_err, say
from workloads.plummer import plummer

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_SRC = r"""
#include <stdio.h>
#include <stdlib.h>
#include <hip/hip_runtime_api.h>
#include "nbody.h"

#define CK(x) do { int _r = (int)(x); if (_r != 0) { fprintf(stderr, "%s failed: %d\n", #x, _r); return 1; } } while (0)

int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "rb");
    long long n; double eps2;
    if (!f || fread(&n, 8, 1, f) != 1 || fread(&eps2, 8, 1, f) != 1) return 2;
    double *h = (double *)malloc(sizeof(double) * 7 * n);
    if (fread(h, 8, 7 * n, f) != (size_t)(7 * n)) return 3;
    fclose(f);
    double *d = NULL;
    /* pos 3n | vel 3n | m n | acc 3n | jerk 3n | pot n | t n | dt n | a 3n | k 3n: 22n */
    CK(hipMalloc((void **)&d, sizeof(double) * 22 * n));
    double *pos = d, *vel = d + 3 * n, *m = d + 6 * n, *acc = d + 7 * n, *jerk = d + 10 * n;
    double *pot = d + 13 * n, *t = d + 14 * n, *dt = d + 15 * n, *a = d + 16 * n, *k = d + 19 * n;
    CK(hipMemcpy(d, h, sizeof(double) * 7 * n, hipMemcpyHostToDevice));
    nbody_ctx *ctx = NULL;
    CK(nbody_create(&ctx, 0, NULL));
    CK(nbody_force(ctx, NULL, n, pos, vel, m, n, eps2, acc, jerk, pot, NBODY_ACC_FP32));
    CK(nbody_sync_status(ctx));
    double *out = (double *)malloc(sizeof(double) * 9 * n);
    CK(hipMemcpy(out, acc, sizeof(double) * 7 * n, hipMemcpyDeviceToHost));
    nbody_system s = {n, t, dt, pos, vel, a, k, m, eps2, 0.02, 0.01, 0.125, 1.0 / (1LL << 40), 0u};
    long long steps = 0, inter = 0;
    CK(nbody_init(ctx, &s, 0.0));
    CK(nbody_blockstep(ctx, &s, 5, 1.0, (int64_t *)&steps, (int64_t *)&inter));
    CK(hipMemcpy(out + 7 * n, t, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
    FILE *g = fopen(argv[2], "wb");
    fwrite(&steps, 8, 1, g);
    fwrite(&inter, 8, 1, g);
    fwrite(out, 8, 9 * n, g);
    fclose(g);
    CK(nbody_destroy(ctx));
    CK(hipFree(d));
    free(h);
    free(out);
    return 0;
}
"""


def test_c_program_calls_the_library_on_the_gpu(orc, tmp_path):
    need_gpu()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib_dir = os.path.join(ROOT, "paper_cs_0702135_amd", "lib")
    src = tmp_path / "prog.c"
    src.write_text(C_SRC)
    exe = tmp_path / "prog"
    cmd = ["gcc", "-std=c99", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe),
           "-L" + lib_dir, "-lnbody", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + lib_dir, "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    n, eps2 = 3001, (1 / 256) ** 2
    pos, vel, m = plummer(n, 91)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.array([n], dtype=np.int64).tofile(f)
        np.array([eps2], dtype=np.float64).tofile(f)
        np.concatenate([pos.ravel(), vel.ravel(), m]).astype(np.float64).tofile(f)
    outp = tmp_path / "out.bin"
    say("C program: n=%d" % n)
    r = subprocess.run([str(exe), str(inp), str(outp)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(outp, dtype=np.int64, count=2)
    steps, inter = int(raw[0]), int(raw[1])
    out = np.fromfile(outp, dtype=np.float64, offset=16)
    acc, jerk, pot = out[:3 * n].reshape(3, n), out[3 * n:6 * n].reshape(3, n), out[6 * n:7 * n]
    t, dt = out[7 * n:8 * n], out[8 * n:9 * n]
    ra, rk, rp = orc.force(pos, vel, m, eps2)
    ea, ek = rel_vec_err(acc, ra), rel_vec_err(jerk, rk)
    say("C program: acc p99 %.2e max %.2e, jerk p99 %.2e, %d block steps, %d interactions"
        % (np.percentile(ea, 99), ea.max(), np.percentile(ek, 99), steps, inter))
    assert np.percentile(ea, 99) <= 1e-6 and ea.max() <= 1e-5
    assert np.percentile(ek, 99) <= 1e-5
    np.testing.assert_allclose(pot, rp, rtol=1e-5)
    assert steps == 5 and inter > 0
    # every particle's time is a multiple of its power-of-two step
    assert np.all(np.fmod(t, dt) == 0) and np.all(np.frexp(dt)[0] == 0.5)
