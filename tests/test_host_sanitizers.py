"""The host runtime (geometry, planning tables, launch selection, argument checks, the
host-only context, the serving scheduler thread through its host test executor) built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven through the C ABI in a
fresh process; any sanitizer report fails the test.  The device
code is compiled as usual (the sanitizers cover the host objects only); no GPU call is
made: the calls run on a host-only context (device -1)."""

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_02292_amd", "csrc")
HOST_SOURCES = ["tomo_plan.cpp", "tomo_capi.cpp", "tomo_serve.cpp", "tomo_local.cpp"]
DEVICE_SOURCES = ["tomo_kernels.hip", "tomo_noalloc.hip", "tomo_probe.hip"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def _build(out):
    from paper_1604_02292_amd.build import COMMON, DEVICE_FLAGS, _hipcc
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out, src + ".o")
        _run(["g++", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + SAN +
             ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"])
        objs.append(obj)
    for src in DEVICE_SOURCES:
        obj = os.path.join(out, src + ".o")
        _run([_hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + ["-x", "hip"] +
             DEVICE_FLAGS)
        objs.append(obj)
    lib = os.path.join(out, "libtomo_san.so")
    _run(["g++", "-shared", "-o", lib] + objs + SAN +
         ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lpthread",
          "-Wl,-rpath,/opt/rocm/lib"])
    return lib


DRIVER = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    from paper_1604_02292_amd import _lib
    _lib.LIB_PATH = {lib!r}
    import synth
    from paper_1604_02292_amd import Context, TomoError, make_params
    ctx = Context(device=-1)
    for n, na, nd in [(128, 32, 192), (97, 45, 150), (2048, 256, 3072), (4096, 512, 6144)]:
        g = ctx.tomo_set_geometry(n, na, nd)
        for rect in [(0, 0, n, n), (0, 0, 1, 1), (n - 7, 3, 7, n - 3), (n // 3, n // 4, 16, 40)]:
            i0, w = ctx.tomo_roi_band(g, rect)
            assert len(i0) == na and min(w) >= 1
            ext = ctx.tomo_roi_ext(g, rect, 9)
            if n <= 2048 and rect[2] * rect[3] <= 4096:
                assert ctx.tomo_roi_nnz(g, rect) > 0
    g3 = ctx.tomo_set_geometry(2048, 256, 3072)
    batch = [make_params(r[:4], r[4], "cp", 0.02, 200) for r in synth.roi_list("c3")]
    print(ctx.tomo_resolve_launch(g3, batch))
    g4 = ctx.tomo_set_geometry(4096, 512, 6144)
    tiles = [make_params(r[:4], r[4], "cp", 0.01, 200) for r in synth.roi_list("c4")]
    print(ctx.tomo_resolve_launch(g4, tiles))
    for knobs in [dict(fp_rays_per_lane=4), dict(fp_segments=8, bp_groups=8), {{}}]:
        ctx.tomo_set_launch(**knobs)
        ctx.tomo_resolve_launch(g3, batch[:5])
    bad = 0
    for kw in [dict(fp_segments=3), dict(fp_rays_per_lane=3), dict(bp_variant=7)]:
        try:
            ctx.tomo_set_launch(**kw)
        except TomoError:
            bad += 1
    assert bad == 3
    for args in [(0, 32, 192), (128, 0, 192), (128, 32, -1)]:
        try:
            ctx.tomo_set_geometry(*args)
            raise AssertionError("accepted " + str(args))
        except TomoError:
            pass
    for rect in [(0, 0, 0, 4), (-1, 0, 4, 4), (120, 120, 16, 16)]:
        try:
            ctx.tomo_roi_band(0, rect)   # the 128-pixel geometry
            raise AssertionError("accepted " + str(rect))
        except TomoError:
            pass
    ctx.close()
    # the serving scheduler (its own thread) through the host test executor, with
    # host buffers passed straight through the C ABI
    import ctypes as C, time
    from paper_1604_02292_amd import _lib as L
    ctx = Context(device=-1)
    lib, h = ctx.lib, ctx.h
    assert lib.tomo_serving_fake(h, 64 << 20, 0) == 0
    assert lib.tomo_serving_config(h, 4, 3) == 0
    g = ctx.tomo_set_geometry(128, 32, 192)
    sino = (C.c_float * (32 * 192))()
    sid = C.c_int32()
    assert lib.tomo_register_sinogram(h, g, C.cast(sino, C.c_void_p), C.byref(sid)) == 0
    outs, tickets = [], []
    for k in range(24):
        out = (C.c_float * 256)()
        p = make_params((10 + k, 20, 16, 16), 4, "cp", 0.05, 3 + k)
        t = C.c_uint64()
        assert lib.roi_submit(h, sid.value, C.byref(p), C.cast(out, C.c_void_p),
                              C.byref(t)) == 0
        outs.append((out, 3 + k))
        tickets.append(t.value)
    pending, t0 = set(tickets), time.time()
    stages = (C.c_float * 4)()
    while pending and time.time() - t0 < 60:
        for t in list(pending):
            done = C.c_int()
            assert lib.roi_poll_stages(h, C.c_uint64(t), C.byref(done), stages) == 0
            if done.value:
                pending.discard(t)
        time.sleep(0.001)
    assert not pending
    for out, it in outs:
        assert all(v == float(it) for v in out)
    assert lib.tomo_synchronize(h) == 0
    assert lib.tomo_unregister_sinogram(h, sid.value) == 0
    # a stalled executor with queued work, ended by destroy
    assert lib.tomo_serving_fake(h, 0, -1) == 0
    assert lib.tomo_register_sinogram(h, g, C.cast(sino, C.c_void_p), C.byref(sid)) == 0
    keep = [(C.c_float * 256)() for _ in range(8)]
    for out in keep:
        p = make_params((40, 40, 16, 16), 4, "cp", 0.05, 50)
        t = C.c_uint64()
        assert lib.roi_submit(h, sid.value, C.byref(p), C.cast(out, C.c_void_p),
                              C.byref(t)) == 0
    ctx.close()
    print("host calls done")
""")


@pytest.mark.timeout(900)
def test_host_runtime_under_address_and_ub_sanitizers(tmp_path):
    lib = _build(str(tmp_path))
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", DRIVER.format(root=ROOT, lib=lib)],
                       capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report, report[-4000:]
    assert "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "host calls done" in r.stdout
