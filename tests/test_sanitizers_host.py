"""Host-side sanitizers (CPU): the library's host code built with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged; the
flags go to the host compilation only), then the host arithmetic of the
method -- power-model fits and bands, tune-space enumeration, selection,
Pareto front, energy from samples, the stale-sensor rule, fitness flow graph,
batch packing, and null/bad-argument error paths -- driven through the C ABI
in a child process with the sanitizer runtime preloaded.  Any memory error or
undefined behaviour aborts the child (recovery is off)."""
import glob
import os
import subprocess
import sys
import textwrap
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2211_07260_amd import build as b  # noqa: E402

pytestmark = pytest.mark.slow

ROCM_LLVM = os.path.join(b.ROCM, "lib", "llvm")
SAN_KINDS = "address," + "undefined"
HOST_SAN = ["-Xarch_host", "-fsanitize=" + SAN_KINDS, "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def asan_runtime():
    hits = glob.glob(os.path.join(ROCM_LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    return hits[0] if hits else None


@pytest.fixture(scope="module")
def san_lib(tmp_path_factory):
    rt = asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this ROCm")
    out = tmp_path_factory.mktemp("san")

    def comp(src):
        obj = str(out / (os.path.basename(src) + ".o"))
        cmd = [b.HIPCC] + b.CFLAGS + HOST_SAN + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    srcs = sorted(glob.glob(os.path.join(b.CSRC, "*.hip")) + glob.glob(os.path.join(b.CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, srcs))
    lib = str(out / "libgreentune.so")
    tlib = b.torch_lib_dir()
    subprocess.run([os.path.join(ROCM_LLVM, "bin", "clang++"), "-shared", "-fPIC", "-fsanitize=" + SAN_KINDS,
                    "-shared-libasan", "-o", lib] + objs +
                   ["-L" + tlib, "-l:libamdhip64.so", "-Wl,-rpath," + tlib, "-L" + os.path.join(b.ROCM, "lib"),
                    "-lamd_smi", "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(b.ROCM, "lib"),
                    "-lpthread"], check=True, capture_output=True)
    return lib, rt


CHILD = textwrap.dedent("""
    import ctypes, sys
    import numpy as np
    sys.path.insert(0, {root!r})
    import paper_2211_07260_amd as gt
    from oracle import power_model as opm
    assert gt.LIB_PATH == {lib!r}
    gt.init(0, gt.INIT_HOST_ONLY)
    rng = np.random.default_rng(0)
    settable = list(np.arange(500.0, 2401.0, 25.0))
    for seed in range(5):
        f = np.linspace(500.0, 2400.0, 5 + seed)
        p = opm.power(f, 200, 0.2, 1e-3, 1200, 1e9) + rng.normal(0, 3, f.size)
        m = gt.fit_power_model(f, p, 1e9)
        gt.fit_power_model(f, p, 1e9, literal=True)
        gt.fit_power_model(f, p, 900.0)
        gt.fit_power_model(f, p, 1e9, v=np.linspace(0.7, 1.1, f.size))
        gt.power_model_band(m, settable)
        gt.power_model_throttle_clock(m)
    gt.power_model_band(gt.power_model(300.0, 0.55, 5e-5, 1500.0, 1400.0), settable)
    prob = gt.xcorr_problem(4096, 4096, 17, 17)
    vals = dict(block_size_x=[16, 32, 64, 128], block_size_y=[1, 2, 4, 8, 16], tile_size_x=list(range(1, 9)),
                tile_size_y=list(range(1, 9)), use_lds_padding=[0, 1], read_path=[0, 1])
    cfgs = gt.tune_space_enumerate(prob, vals, lds_limit=163840)
    assert len(cfgs) == 3572
    recs = [dict(t_run_s=float(rng.uniform(1, 2)), e_run_j=float(rng.uniform(1, 2))) for _ in range(200)]
    gt.select(recs, "time"); gt.select(recs, "energy"); gt.pareto(recs); gt.pareto(recs[:1])
    t = np.sort(rng.uniform(0, 1, 500)); pw = rng.uniform(900, 1100, 500)
    gt.energy_from_samples(t, pw, 0.1, 0.9, 1000, 0.2)
    try:  # two readings that may both lie outside the kept window
        gt.energy_from_samples(t[:2], pw[:2], 0.1, 0.9, 1, 0.0)
    except gt.GreentuneError as e:
        assert e.code == gt.GT_E_SENSOR
    gt.sensor_stale(t, pw); gt.sensor_stale(t[:1], pw[:1])
    gt.ffg_centrality([tuple(c.as_tuple()) for c in cfgs[:300]], rng.lognormal(0, 0.3, 300))
    lib = gt.lib()
    assert lib.fit_power_model(None, None, None, 0, 1.0, None) == gt.GT_E_INVAL
    assert lib.gt_select(None, 0, 0, None) == gt.GT_E_INVAL
    assert lib.gt_pareto(None, 3, None) == gt.GT_E_INVAL
    assert lib.tune_space_enumerate(None, None, None, 0, None) == gt.GT_E_INVAL
    items = (gt.BatchItem * 3)(*[gt.BatchItem(0x1000 * (k + 1), 0x20000, 0x30000, 10 + k, 20, 5, 5) for k in range(3)])
    nb, tt = ctypes.c_size_t(0), ctypes.c_int64(0)
    cfg = gt.as_config((32, 8, 4, 4, 0, 0))
    assert lib.gt_batch_pack(items, 3, ctypes.byref(cfg), None, 0, ctypes.byref(nb), ctypes.byref(tt)) == gt.GT_E_CAPACITY
    blob = (ctypes.c_uint8 * nb.value)()
    assert lib.gt_batch_pack(items, 3, ctypes.byref(cfg), blob, nb.value, ctypes.byref(nb), ctypes.byref(tt)) == 0
    shape = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, 1, 1, 32, 32, 5, 5)
    assert lib.gt_igemm_batch_pack(ctypes.byref(shape), items, 3, None, 0, ctypes.byref(nb),
                                   ctypes.byref(tt)) == gt.GT_E_CAPACITY
    assert lib.conv2d_run_batched_noalloc(items, 5000, ctypes.byref(cfg), 0, None) == gt.GT_E_INVAL
    gt.shutdown()
    print("host calls ok", flush=True)
""")


def test_host_code_under_asan_and_ubsan(san_lib):
    lib, rt = san_lib
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in nm and "__ubsan_handle" in nm   # the host code is instrumented
    env = dict(os.environ, GREENTUNE_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env, capture_output=True,
                       text=True, timeout=600)
    report = p.stdout[-3000:] + p.stderr[-6000:]
    assert p.returncode == 0, report
    assert "host calls ok" in p.stdout
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
