"""CPU checks of the C ABI: the header compiles as C, the library loads and
exports every declared entry point, and host-side validation rejects bad
arguments before anything touches a GPU."""
import ctypes
import os
import re
import subprocess

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_compiles_as_c_and_cpp():
    for std, lang in (("c11", "c"), ("c++17", "c++")):
        r = subprocess.run(["gcc", "-x", lang, f"-std={std}", "-fsyntax-only", "-Wall", "-Werror", HEADER],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("dgsm_build", "dgsm_query", "sh_transfer", "dgsm_build_workspace_size",
              "dgsm_status_string", "dgsm_alpha_centroid"):
        assert n in names


@pytest.fixture(scope="module")
def lib():
    import paper_2601_01660_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libdgsm.so not built")
    return P.lib()


def test_library_exports_every_declared_symbol(lib):
    r = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True)
    exported = set(line.split()[-1] for line in r.stdout.splitlines() if line.strip())
    for n in declared_functions():
        assert n in exported, n
        assert hasattr(lib, n)


def test_status_strings(lib):
    import paper_2601_01660_amd as P
    for s in range(5):
        assert isinstance(lib.dgsm_status_string(s), bytes)
    assert P.lib().dgsm_status_string(0) == b"ok"


# Tests below hand the library fake device pointers (1, 1 << 40) and rely on
# host-side validation returning before anything is enqueued.  That holds by
# construction, but such a pointer must never get near a real device, so they
# run only where no GPU is visible.
fake_pointers = pytest.mark.skipif(torch.cuda.is_available(),
                                   reason="passes fake device pointers; host-only check")


def _desc(**kw):
    import paper_2601_01660_amd as P
    base = dict(H=32, W=32, K=16, spacing="geometric", r0=0.05, r1=8.0, dtype="f32", cull_eps=1e-8)
    base.update(kw)
    return P.Atlas(**base)


def test_workspace_size_is_host_only_and_grows_with_n(lib):
    import paper_2601_01660_amd as P
    a = P.dgsm_build_workspace_size(_desc(), 0, 1)
    b = P.dgsm_build_workspace_size(_desc(), 5000, 1)
    c = P.dgsm_build_workspace_size(_desc(H=512, W=512, K=64), 2_150_000, 4)
    assert 0 < a < b < c


@fake_pointers
@pytest.mark.parametrize("bad", [dict(H=31), dict(W=0), dict(K=1), dict(K=513), dict(r0=0.0),
                                 dict(r0=9.0), dict(r1=-1.0), dict(cull_eps=-1.0)])
def test_invalid_descriptions_are_rejected(lib, bad):
    import paper_2601_01660_amd as P
    assert P.dgsm_build_workspace_size(_desc(**bad), 10, 1) == 0
    d = _desc(**bad).struct()
    lt = P._Lights(1, 1, 1.0)          # never dereferenced: validation comes first
    gs = P._Gaussians(0, 0, 0, 0, 0)
    st = lib.dgsm_build(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), 1, 1, 1 << 40, None)
    assert st == 1


@pytest.mark.parametrize("H,W,ok", [(32, 48, True), (4, 6, True), (30, 45, True), (2, 3, False),
                                     (32, 32, False), (48, 32, False), (31, 46, False)])
def test_cube_map_descriptions(lib, H, W, ok):
    import paper_2601_01660_amd as P
    assert (P.dgsm_build_workspace_size(_desc(H=H, W=W, param="cubemap"), 10, 1) > 0) == ok


@fake_pointers
def test_unknown_parameterisation_and_cube_map_learned_field_are_rejected(lib):
    import paper_2601_01660_amd as P
    d = _desc().struct()
    d.param = 7
    assert lib.dgsm_build_workspace_size(ctypes.byref(d), 10, 1) == 0
    cube = _desc(H=32, W=48, param="cubemap").struct()
    stats = (ctypes.c_uint32 * 4)()
    # validation comes first: the device pointers are never dereferenced
    st = lib.dgsm_mlp_check(1, ctypes.byref(cube), 1, 16, 1, ctypes.c_float(0.01), 1, stats, 1, 1 << 40, None)
    assert st == 4
    octa = _desc().struct()
    st = lib.dgsm_mlp_check(1, ctypes.byref(octa), 1, 16, 1, ctypes.c_float(0.01), 1, stats, 1, 16, None)
    assert st == 2                         # octahedral passes, then the workspace is too small


@fake_pointers
def test_null_pointers_and_small_workspace_are_rejected(lib):
    import paper_2601_01660_amd as P
    d = _desc().struct()
    gs = P._Gaussians(0, 0, 0, 0, 5)          # n > 0 with null arrays
    lt = P._Lights(1, 1, 1.0)
    assert lib.dgsm_build(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), 1, 1, 1 << 40, None) == 1
    gs = P._Gaussians(1, 1, 1, 1, 5)
    assert lib.dgsm_build(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), 1, 1, 16, None) == 2
    assert lib.dgsm_build(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), 1, None, 1 << 40, None) == 2
    lt0 = P._Lights(0, 1, 1.0)
    assert lib.dgsm_build(ctypes.byref(lt0), ctypes.byref(gs), ctypes.byref(d), 1, 1, 1 << 40, None) == 1
    assert lib.dgsm_query(ctypes.byref(lt), ctypes.byref(d), None, 1, 10, 1, None) == 1
    prm = P._ShParams(32, 64, 1.0, 4.0, 1e-6, 1.0, 0)
    ws = 1 << 20
    assert lib.sh_transfer(1, 16, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, None, 1, ws, None) == 1
    prm = P._ShParams(32, 64, 1.0, 4.0, 1e-6, 1.0, 1)
    assert lib.sh_transfer(1, 5, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, None, 1, ws, None) == 1
    assert lib.sh_transfer(1, 16, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, 1, 1, ws, None) == 1
    assert lib.sh_transfer(1, 16, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, None, 1, 64, None) == 2
    assert lib.sh_transfer(1, 16, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, None, None, ws, None) == 2
    # the probe table is written with 16-byte stores: a misaligned workspace is refused
    assert lib.sh_transfer(1, 16, ctypes.byref(gs), None, ctypes.byref(prm), 1, None, None, 8, ws, None) == 1


def test_sh_workspace_covers_the_padded_grid(lib):
    """16 bytes per direction of the grid with its columns padded to a
    multiple of 16, then the cosines and sines of the 16 columns of a group,
    of the groups' first edges (at least two) and of the rows, each part
    256-byte aligned."""
    up = lambda b: (b + 255) // 256 * 256
    for nt, nph in ((32, 64), (7, 13), (1, 1), (48, 100), (4, 2048)):
        p16 = (nph + 15) // 16 * 16
        want = up(nt * p16 * 16) + up(16 * 8) + up(max(2, p16 // 16) * 8) + up(nt * 8)
        assert lib.sh_transfer_workspace_size(nt, nph) == want
    assert lib.sh_transfer_workspace_size(0, 64) == 0
    assert lib.sh_transfer_workspace_size(1 << 12, 1 << 13) == 0


@fake_pointers
def test_noalloc_build_validates_and_refuses_oversized_requests_first(lib):
    import paper_2601_01660_amd as P
    assert lib.dgsm_build_noalloc_max_bytes() == 64 * 1024 * 1024
    d = _desc().struct()
    lt = P._Lights(1, 1, 1.0)
    gs = P._Gaussians(0, 0, 0, 0, 5)          # n > 0 with null arrays
    assert lib.dgsm_build_noalloc(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), 1, None) == 1
    gs = P._Gaussians(1, 1, 1, 1, 5)
    assert lib.dgsm_build_noalloc(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), None, None) == 1
    big = _desc(H=512, W=512, K=64).struct()
    gs = P._Gaussians(1, 1, 1, 1, 2_000_000)
    assert lib.dgsm_build_workspace_size(ctypes.byref(big), 2_000_000, 1) > lib.dgsm_build_noalloc_max_bytes()
    assert lib.dgsm_build_noalloc(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(big), 1, None) == 2


@fake_pointers
def test_check_and_work_unit_queries_validate_first(lib):
    import paper_2601_01660_amd as P
    n_bad = ctypes.c_longlong(-1)
    gs = P._Gaussians(0, 0, 0, 0, 5)          # n > 0 with null arrays
    assert lib.dgsm_check_gaussians(ctypes.byref(gs), 1, ctypes.byref(n_bad), None) == 1
    gs = P._Gaussians(1, 1, 1, 1, 5)
    assert lib.dgsm_check_gaussians(ctypes.byref(gs), None, ctypes.byref(n_bad), None) == 1
    assert lib.dgsm_check_gaussians(ctypes.byref(gs), 1, None, None) == 1
    d = _desc().struct()
    out = (ctypes.c_int32 * 4)()
    assert lib.dgsm_work_units(ctypes.byref(d), 100, 2, 1, 16, 0, out, None) == 2       # workspace too small
    assert lib.dgsm_work_units(ctypes.byref(d), 100, 2, 1, 1 << 40, 2, out, None) == 1  # light out of range
    assert n_bad.value == -1


def test_binding_rejects_host_tensors_for_device_arguments():
    """A host pointer must never reach a kernel: the binding refuses CPU tensors
    where the library expects device memory."""
    import torch
    import paper_2601_01660_amd as P
    g = P.GaussianSet(torch.zeros(4, 3), torch.ones(4, 3), torch.zeros(4, 4), torch.zeros(4))
    with pytest.raises(ValueError):
        g.struct()
    with pytest.raises(ValueError):
        P._cuda(torch.zeros(3), "x")
    assert P._cuda(None, "x") is None


def test_binding_shape_helpers():
    """[n, 3] inputs and exactly-sized buffers are checked before any call."""
    import torch
    import paper_2601_01660_amd as P
    assert P._rows(torch.zeros(5, 3), 3, "points").shape == (5, 3)
    for bad in (torch.zeros(5), torch.zeros(5, 4), torch.zeros(2, 5, 3)):
        with pytest.raises(ValueError):
            P._rows(bad, 3, "points")
    with pytest.raises(ValueError):
        P._buf(torch.zeros(2, 3), (2, 3), torch.float32, "out")     # host tensor
    assert P._buf(None, (2, 3), torch.float32, "out") is None


def test_library_stencil_matches_the_oracle_reading(lib):
    import numpy as np
    import paper_2601_01660_amd as P
    from oracle import dgsm as od
    z, w = P.dgsm_footprint_stencil7()
    zo, wo = od.footprint_stencil7()
    assert np.array_equal(z.numpy(), zo.astype(np.float32))
    assert np.allclose(w.numpy(), wo, rtol=0, atol=1e-7)


@fake_pointers
def test_footprint_query_validates_sample_count(lib):
    import paper_2601_01660_amd as P
    d = _desc().struct()
    lt = P._Lights(1, 1, 1.0)
    gs = P._Gaussians(1, 1, 1, 1, 5)
    assert lib.dgsm_query_footprint(ctypes.byref(lt), ctypes.byref(d), 1, ctypes.byref(gs), 1, 1, 0, 1, None) == 1
    assert lib.dgsm_query_footprint(ctypes.byref(lt), ctypes.byref(d), 1, ctypes.byref(gs), 1, 1, 65, 1, None) == 1
    assert lib.dgsm_query_footprint(ctypes.byref(lt), ctypes.byref(d), 1, ctypes.byref(gs), None, 1, 7, 1, None) == 1


def test_gaussian_set_arrays_must_match_the_mean_count():
    """Every array of a Gaussian set is checked against N = mean.shape[0] before
    any pointer is handed over (the kernels read 3, 3, 4 and 1 floats per Gaussian)."""
    import paper_2601_01660_amd as P
    n = 6
    good = dict(mean=torch.zeros(n, 3), scale=torch.ones(n, 3), rot=torch.zeros(n, 4), opacity=torch.zeros(n))
    bad_cases = [dict(scale=torch.ones(n - 1, 3)), dict(scale=torch.ones(n, 2)), dict(rot=torch.zeros(n, 3)),
                 dict(rot=torch.zeros(n + 1, 4)), dict(opacity=torch.zeros(n, 1)), dict(opacity=torch.zeros(n - 2)),
                 dict(mean=torch.zeros(n, 4)), dict(mean=torch.zeros(3 * n))]
    for bad in bad_cases:
        kw = dict(good, **bad)
        with pytest.raises(ValueError, match="shape"):
            P.GaussianSet(**kw).struct()
    with pytest.raises(ValueError, match="float32"):
        P.GaussianSet(**dict(good, opacity=torch.zeros(n, dtype=torch.float64))).struct()
    # right shapes on the host: refused as host memory, not for their shapes
    with pytest.raises(ValueError, match="CUDA"):
        P.GaussianSet(**good).struct()


def test_sh_transfer_checks_probe_colour_and_centroid_shapes():
    import paper_2601_01660_amd as P
    n = 5
    gs = P.GaussianSet(torch.zeros(n, 3), torch.ones(n, 3), torch.zeros(n, 4), torch.zeros(n))
    probe = torch.zeros(16, 3)
    for bad_probe in (torch.zeros(8, 3), torch.zeros(16, 4), torch.zeros(48), torch.zeros(25, 3)):
        with pytest.raises(ValueError, match="probe_sh"):
            P.sh_transfer(bad_probe, gs)
    for bad_colour in (torch.zeros(n, 9, 3), torch.zeros(n - 1, 16, 3), torch.zeros(n, 48)):
        with pytest.raises(ValueError, match="colour_sh"):
            P.sh_transfer(probe, gs, colour_sh=bad_colour)
    for bad_c in (torch.zeros(2), torch.zeros(1, 3), torch.zeros(4)):
        with pytest.raises(ValueError, match="centroid"):
            P.sh_transfer(probe, gs, centroid=bad_c)
    for kp in (1, 4, 9, 16):        # accepted shapes get as far as the host-memory check
        with pytest.raises(ValueError, match="CUDA"):
            P.sh_transfer(torch.zeros(kp, 3), gs, colour_sh=torch.zeros(n, 16, 3), centroid=torch.zeros(3))


def test_mlp_checkpoint_round_trip(lib, tmp_path):
    """Parameters, Adam moments, step and atlas geometry survive a save/load
    bit for bit; the header is the documented JSON line; a file without moments
    cannot fill a request for them, and a foreign file is refused."""
    import json

    import numpy as np

    import paper_2601_01660_amd as P
    rng = np.random.default_rng(3)
    params = torch.from_numpy(rng.standard_normal(P.MLP_PARAMS).astype(np.float32))
    adam = torch.from_numpy(rng.standard_normal(2 * P.MLP_PARAMS).astype(np.float32))
    atlas = P.Atlas(512, 384, 64, spacing="geometric", r0=0.05, r1=8.0)
    path = str(tmp_path / "light0.dgsm")
    P.mlp_save(path, params, atlas, adam_mv=adam, step=1500)
    p2, m2, step, a2 = P.mlp_load(path)
    assert torch.equal(p2, params) and torch.equal(m2, adam) and step == 1500
    assert (a2.H, a2.W, a2.K, a2.spacing) == (512, 384, 64, "geometric")
    assert a2.r0 == np.float32(0.05) and a2.r1 == np.float32(8.0)
    with open(path, "rb") as f:
        assert f.readline() == b"DGSM-MLP 1\n"
        head = json.loads(f.readline())
        body = f.read()
    assert head["params"] == P.MLP_PARAMS and head["adam"] == 1 and head["step"] == 1500
    assert len(body) == 3 * 4 * P.MLP_PARAMS
    assert np.array_equal(np.frombuffer(body[:4 * P.MLP_PARAMS], "<f4"), params.numpy())
    # parameters only
    path2 = str(tmp_path / "light1.dgsm")
    P.mlp_save(path2, params, atlas, step=7)
    p3, m3, step3, _ = P.mlp_load(path2, adam=False)
    assert torch.equal(p3, params) and m3 is None and step3 == 7
    with pytest.raises(P.DGSMError):
        P.mlp_load(path2, adam=True)
    bad = tmp_path / "bad.dgsm"
    bad.write_bytes(b"not a checkpoint\n{}\n")
    with pytest.raises(P.DGSMError):
        P.mlp_load(str(bad))
    with pytest.raises(P.DGSMError):
        P.mlp_load(str(tmp_path / "missing.dgsm"))


def test_host_paths_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The library's host code (argument validation, workspace sizing,
    checkpoint parsing) built with ASan and UBSan on the host pass only and
    driven by tests/abi_sanitize.cpp: every invalid call returns its status
    without a sanitizer report.  Device code is compiled as usual."""
    import sys
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or torch.cuda.is_available():
        pytest.skip("host-only sanitizer build (runs where hipcc is present and no GPU is visible)")
    sys.path.insert(0, ROOT)
    from paper_2601_01660_amd import build as b
    exe = str(tmp_path / "abi_sanitize")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [hipcc, *b.HIPCC_FLAGS, *san, "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2601_01660_amd", "csrc"), *b.sources(),
           os.path.join(ROOT, "tests", "abi_sanitize.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower() and "not found" in (r.stderr + r.stdout):
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
