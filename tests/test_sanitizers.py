"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: the host library
(plan validation, image enumeration, delay blocks and groups, tables, error
predictions, everything msim_plan_create does before it needs a device) and the
oracle, each built with the sanitizers and driven in a child process that
preloads the matching runtime.  Any report fails the test (the runtimes halt on
the first one).  The sanitized builds are kept beside the regular ones
(git-ignored) and rebuilt when their sources change."""
import glob
import hashlib
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2508_03065_amd")


def _sources_sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _cached_build(out, files, make):
    stamp = out + ".sha"
    sha = _sources_sha(files)
    if not (os.path.exists(out) and os.path.exists(stamp) and open(stamp).read() == sha):
        make(out)
        with open(stamp, "w") as f:
            f.write(sha)
    return out


def _run(script, preload, extra_env=None):
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    env.update(extra_env or {})
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return r.stdout


def test_host_library_under_asan_ubsan():
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang ASan runtime not found")
    from paper_2508_03065_amd import build
    srcs = sorted(glob.glob(os.path.join(PKG, "csrc", "*"))) + [os.path.join(ROOT, "include", "msim.h")]
    lib = _cached_build(os.path.join(PKG, "libmsim_san.so"), srcs,
                        lambda out: build.build(sanitize=True, out=out))
    out = _run("""
        import ctypes as C, dataclasses, sys
        sys.path.insert(0, %r)
        from paper_2508_03065_amd import _lib, scenegen as G
        from paper_2508_03065_amd.msim import params_struct, Plan
        _lib.LIB_PATH = %r
        L = _lib.load()
        n = C.c_int64()
        for K in range(0, 25):
            assert L.msim_count_images(K, C.byref(n)) == 0
        cases = [G.config1(), G.config2(seconds=1.0), G.config4(), G.config5(n_scenes=1, seconds=1.0)]
        s3, p3 = G.config3()
        cases.append((s3[:8], p3))
        e2 = getattr(G, "e2_scenes", None)
        if e2 is not None:
            cases.append(e2(n_scenes=2, seed=3)[:2])
        codes = []
        for scenes, par in cases:
            for fd in (0, 1):
                for slack in (0.0, 0.05):
                    p = dataclasses.replace(par, fd_kind=fd, knot_slack=slack)
                    try:
                        Plan(scenes, p)
                        codes.append("ok")
                    except _lib.MsimError as e:
                        codes.append(str(e).split(":")[0])
        # refusals: table error above budget, bad params
        sc, par = G.small_scene(seed=1, taps=32)
        for mut in (dict(kaiser_beta=0.0, cutoff=0.5), dict(cutoff=0.7), dict(taps=40)):
            try:
                Plan([sc], dataclasses.replace(par, **mut), table_phases=64)
            except _lib.MsimError as e:
                codes.append(str(e).split(":")[0])
        print("codes", codes)
    """ % (ROOT, lib), rt[0])
    assert "codes" in out
    # without a device every valid plan stops at the device query, after all host work
    assert "MSIM_E_HIP" in out and "MSIM_E_UNSUPPORTED" in out and "MSIM_E_INVALID_ARG" in out


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc ASan runtime not found")
    src = os.path.join(ROOT, "oracle", "msim_oracle.c")
    lib = _cached_build(os.path.join(ROOT, "oracle", "liboracle_san.so"), [src], lambda out: subprocess.check_call(
        ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-o", out, src, "-lm"]))
    script = """
        import dataclasses, sys, numpy as np
        sys.path.insert(0, %r)
        from oracle import oracle as O
        from paper_2508_03065_amd import scenegen as G
        O.LIB = %r
        sc, par = G.small_scene(seed=5, max_order=3, seconds=0.05, taps=32, n_mics=2, moving_rcv=True,
                                tiers=((1, 1), (2, 4), (99, 16)))
        c, par_c = G.small_scene(seed=6, max_order=2, seconds=0.04, taps=64, circle=True)
        res = []
        for s, ps in ((sc, par), (c, par_c)):
            for model in (0, 1):
                p = dataclasses.replace(ps, delay_model=model)
                y = O.forward(s, p)
                gy = np.random.default_rng(1).standard_normal(y.shape)
                res += [y.sum(), O.forward(s, p, idx=[0, 5, 17]).sum(), O.adjoint_x(s, p, gy).sum(),
                        O.grad_beta(s, p, gy).sum(), O.forward(s, dataclasses.replace(p, tiers=())).sum()]
        print("sums", repr([float(v) for v in res]))
    """ % (ROOT, lib)
    san = _run(script, asan)
    # the same numbers from the regular build (no preload)
    ref = subprocess.run([sys.executable, "-c", textwrap.dedent(script.replace("O.LIB = %r" % lib, ""))],
                         capture_output=True, text=True, timeout=600, cwd=ROOT, env=dict(os.environ, OMP_NUM_THREADS="4"))
    assert ref.returncode == 0, ref.stderr[-2000:]
    a = eval(san.strip().splitlines()[-1][5:])
    b = eval(ref.stdout.strip().splitlines()[-1][5:])
    # the same values up to the order of the oracle's threaded sums
    assert len(a) == len(b) and all(abs(u - v) <= 1e-12 * max(1.0, abs(v)) for u, v in zip(a, b)), (a, b)
