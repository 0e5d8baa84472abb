"""The C-ABI library loads, exports every declared entry point and rejects bad
arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2405_00366_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "l0cim.h")

FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(l0cim_[a-z0-9_]+)\s*\(", text)))


def test_library_built_and_exports_every_declared_symbol():
    assert os.path.exists(L.library_path), "build with python paper_2405_00366_amd/build.py"
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in l0cim.h but not exported"


def test_version_and_status_strings():
    lib = L.lib()
    assert lib.l0cim_version() == 100
    assert lib.l0cim_status_string(0) == b"ok"
    assert lib.l0cim_status_string(3).startswith(b"workspace")


def test_paper_default_parameters():
    p = L.cim_params()
    assert (p.dt, p.n_steps, p.p_thr, p.d, p.t_c, p.t_w, p.K, p.tau) == (0.02, 1000, 1.0, 0.4, 4.0, 2.0, 1.0, 1.0)
    assert p.c0_std == 1e-2 and p.field == L.FIELD_CN
    s = L.solve_params()
    assert (s.eta_init, s.eta_end, s.velo, s.cdp_iters, s.dtc) == (0.8, 0.18, 51, 100, 0.1)


def test_struct_layouts_match_header():
    assert ctypes.sizeof(L.CimParams) == 104
    assert ctypes.sizeof(L.SolveParams) == 64
    assert ctypes.sizeof(L.Stats) == 40


def test_workspace_sizes():
    lib = L.lib()
    cim, sp = L.cim_params(), L.solve_params()
    ws = lib.l0cim_solve_workspace_bytes(L.F32, 1000, 2000, ctypes.byref(cim), ctypes.byref(sp))
    # G and J take 2 * 2000^2 * 4 bytes; the matrix-core run's panel copy of
    # J (2000 x 2016 x 4), the FP64 Cholesky refit's padded factor (2048^2 x 8)
    # and the CDP's compacted support block (at most 2000^2 x 4) come on top
    assert 32_000_000 <= ws < 32_000_000 + 2000 * 2016 * 4 + 2048 * 2048 * 8 + 2000 * 2000 * 4 + 4_000_000
    assert lib.l0cim_mfcim_run_workspace_bytes(L.F32, 2000, 1, L.F32) >= 2 * 2000 * 8
    assert lib.l0cim_mfcim_run_workspace_bytes(L.F64, 2000, 1, L.F64) >= 2 * 2000 * 16
    assert lib.l0cim_update_r_workspace_bytes(L.F64, 100, L.CDP_CHOL_F64) >= 100 * 100 * 8
    assert lib.l0cim_solve_workspace_bytes(L.F32, 0, 10, ctypes.byref(cim), ctypes.byref(sp)) == 0


def _err(lib):
    return lib.l0cim_last_error().decode()


def test_gram_rejects_bad_arguments_on_host():
    lib = L.lib()
    assert lib.l0cim_gram(L.F32, 4, 4, None, 4, FAKE, FAKE, 4, FAKE, None) == 1
    assert "NULL" in _err(lib)
    assert lib.l0cim_gram(L.F32, 4, 4, FAKE, 3, FAKE, FAKE, 4, FAKE, None) == 2
    assert lib.l0cim_gram(L.F32, 0, 4, FAKE, 4, FAKE, FAKE, 4, FAKE, None) == 2
    assert lib.l0cim_gram(L.BF16, 4, 4, FAKE, 4, FAKE, FAKE, 4, FAKE, None) == 5


def test_init_r_rejects_bad_arguments_on_host():
    lib = L.lib()
    assert lib.l0cim_init_r(L.F32, 4, None, 4, FAKE, FAKE, None, None, None) == 1
    assert "NULL" in _err(lib)
    assert lib.l0cim_init_r(L.F32, 4, FAKE, 3, FAKE, FAKE, None, None, None) == 2
    assert lib.l0cim_init_r(L.F64, 0, FAKE, 4, FAKE, FAKE, None, None, None) == 2
    assert lib.l0cim_init_r(L.FP8E4M3, 4, FAKE, 4, FAKE, FAKE, None, None, None) == 5


def test_mri_run_rejects_bad_arguments_on_host():
    lib = L.lib()
    prm = L.cim_params()
    call = lambda size=128, levels=3, P=2, mask=FAKE, ts=0, tr=None, gamma=0.0: lib.l0cim_mri_mfcim_run(
        size, levels, P, mask, FAKE, FAKE, 1, FAKE, gamma, 0.1, ctypes.byref(prm), FAKE, FAKE, FAKE, None, tr, ts,
        None, None)
    assert call(mask=None) == 1
    assert call(P=0) == 2
    assert call(levels=8) == 2
    assert call(levels=40) == 2
    assert call(levels=-1) == 2
    assert call(ts=5) == 1
    assert call(gamma=-1.0) == 1
    assert call(size=64) == 5          # the 128 x 128 image only


def test_mri_pipeline_entry_points_reject_bad_arguments_on_host():
    lib = L.lib()
    assert lib.l0cim_mri_l2_diag(128, 3, 1e-4, None, 1, FAKE, None) == 1
    assert lib.l0cim_mri_l2_diag(128, 8, 1e-4, FAKE, 1, FAKE, None) == 2
    assert lib.l0cim_mri_l2_diag(64, 3, 1e-4, FAKE, 1, FAKE, None) == 5
    assert lib.l0cim_mri_l2_diag(128, 3, -1.0, FAKE, 1, FAKE, None) == 1
    assert lib.l0cim_mri_lasso(128, 3, 1e-4, FAKE, FAKE, 3e-4, -1, FAKE, None) == 1
    assert lib.l0cim_mri_lasso(128, 3, 1e-4, None, FAKE, 3e-4, 10, FAKE, None) == 1
    upd = lambda cdp=L.CDP_CG, iters=100, cg_max=100, tol=1e-5: lib.l0cim_mri_update_r(
        128, 3, 1e-4, FAKE, FAKE, 1, FAKE, FAKE, cdp, 0.1, iters, cg_max, tol, FAKE, None, None, None)
    assert upd(cdp=L.CDP_CHOL_F64) == 5
    assert upd(cdp=L.CDP_JACOBI, iters=-1) == 1
    assert upd(cg_max=-1) == 1
    assert upd(tol=-1.0) == 1
    mp, cim, sp = L.mri_params(), L.cim_params(), L.solve_params(replicas=2)
    assert lib.l0cim_mri_solve_workspace_bytes(4915, 64, 0) > 64 * 16384 * 9
    assert lib.l0cim_mri_solve_workspace_bytes(0, 64, 0) == 0
    solve = lambda mp=mp, sp=sp, ws=FAKE, nbytes=1 << 40, m=10: lib.l0cim_mri_solve(
        ctypes.byref(mp), m, FAKE, 16384, FAKE, FAKE, ctypes.byref(cim), ctypes.byref(sp), FAKE, FAKE, FAKE, ws,
        nbytes, None)
    assert solve(ws=None) == 3
    assert solve(nbytes=10) == 3
    assert solve(m=0) == 2
    assert solve(mp=L.mri_params(cdp=L.CDP_CHOL_F64)) == 5
    assert solve(mp=L.mri_params(gamma=1e-4), sp=L.solve_params(replicas=2, final_refit_f64=1)) == 5
    assert solve(sp=L.solve_params(replicas=0)) == 1
    assert lib.l0cim_mri_solve_many_workspace_bytes(4, 4915, 64, 0) > 4 * 64 * 16384 * 9
    assert lib.l0cim_mri_solve_many_workspace_bytes(0, 4915, 64, 0) == 0
    seeds = (ctypes.c_uint64 * 4)(1, 2, 3, 4)
    many = lambda count=4, sA=10 * 16384, sy=10, sm=16384, sd=seeds, ws=FAKE, nbytes=1 << 40: \
        lib.l0cim_mri_solve_many(ctypes.byref(mp), count, 10, FAKE, 16384, sA, FAKE, sy, FAKE, sm,
                                 ctypes.cast(sd, ctypes.c_void_p) if sd is not None else None, ctypes.byref(cim),
                                 ctypes.byref(sp), FAKE, FAKE, FAKE, ws, nbytes, None)
    assert many(sd=None) == 1
    assert many(count=0) == 1
    assert many(sA=-1) == 2 and many(sA=5) == 2
    assert many(sy=9) == 2
    assert many(sm=100) == 2
    assert many(ws=None) == 3 and many(nbytes=10) == 3


def test_couplings_rejects_bad_arguments_on_host():
    lib = L.lib()
    # FP8 storage needs row scales
    assert lib.l0cim_build_couplings(L.F32, 8, FAKE, 8, FAKE, FAKE, L.FP8E4M3, FAKE, 8, None, FAKE, None) == 1
    # FP64 arithmetic cannot store BF16
    assert lib.l0cim_build_couplings(L.F64, 8, FAKE, 8, FAKE, FAKE, L.BF16, FAKE, 8, FAKE, FAKE, None) == 5
    assert lib.l0cim_build_couplings(L.F32, 8, FAKE, 8, FAKE, FAKE, L.F32, FAKE, 7, None, FAKE, None) == 2


def test_mfcim_run_rejects_bad_arguments_on_host():
    lib = L.lib()
    prm = L.cim_params()
    args = lambda **kw: dict(dt=L.F32, n=16, P=1, jdt=L.F32, J=FAKE, ldj=16, rs=None, z=FAKE, eta=0.5,
                             prm=ctypes.byref(prm), c=FAKE, e=FAKE, sig=FAKE, H=None, tr=None, ts=0,
                             st=None, ws=FAKE, wsb=1 << 20, s=None) | kw

    def call(a):
        return lib.l0cim_mfcim_run(*a.values())

    assert call(args(wsb=16)) == 3
    assert call(args(ws=None)) == 3
    assert call(args(ldj=15)) == 2
    assert call(args(P=0)) == 2
    assert call(args(ts=5)) == 1                    # trace_steps without a buffer
    bad = L.cim_params(field=7)
    assert call(args(prm=ctypes.byref(bad))) == 1
    bad = L.cim_params(dt=0.0)
    assert call(args(prm=ctypes.byref(bad))) == 1
    bad = L.cim_params(launch=9)
    assert call(args(prm=ctypes.byref(bad))) == 1


def test_solve_rejects_bad_arguments_on_host():
    lib = L.lib()
    cim, sp = L.cim_params(), L.solve_params(n_outer=3, velo=3)
    base = [L.F32, 10, 20, FAKE, 20, FAKE, None, ctypes.byref(cim), ctypes.byref(sp), FAKE, FAKE, FAKE,
            FAKE, 1 << 30, None]
    a = list(base)
    a[13] = 1024
    assert lib.l0cim_solve(*a) == 3
    a = list(base)
    a[4] = 19
    assert lib.l0cim_solve(*a) == 2
    sp0 = L.solve_params(replicas=0)
    a = list(base)
    a[8] = ctypes.byref(sp0)
    assert lib.l0cim_solve(*a) == 1
    sp1 = L.solve_params(j_dtype=L.BF16)
    a = list(base)
    a[0] = L.F64
    a[8] = ctypes.byref(sp1)
    assert lib.l0cim_solve(*a) == 5


def test_update_r_rejects_bad_arguments_on_host():
    lib = L.lib()
    assert lib.l0cim_update_r(L.F32, 10, FAKE, 10, FAKE, FAKE, 7, 0.1, 100, FAKE, None, FAKE, 1 << 20, None) == 1
    assert lib.l0cim_update_r(L.F32, 10, FAKE, 10, FAKE, FAKE, 0, 0.1, -1, FAKE, None, FAKE, 1 << 20, None) == 1
    assert lib.l0cim_update_r(L.F32, 10, FAKE, 10, FAKE, FAKE, 1, 0.1, 0, FAKE, None, FAKE, 64, None) == 3


def _al(x):
    return (x + 255) // 256 * 256


def test_server_footprint_formula():
    """Per-request arena bytes: G and compacted G (n x ld), J (n padded to 16
    x ld), four per-spin vectors and sigma (ld), three P x ld state arrays,
    two P x ld support-bit arrays, P x n supports and energy terms, the CDP
    scratch, and the copies of A and y; every array 256-byte aligned."""
    lib = L.lib()
    for (m, n, P, jdt, jb) in [(50, 96, 8, L.F32, 4), (4915, 8192, 8, L.BF16, 2), (7, 33, 64, L.FP8E4M3, 1)]:
        sp = L.solve_params(replicas=P, j_dtype=jdt)
        ld = (n + 31) // 32 * 32
        n16 = (n + 15) // 16 * 16
        want = (2 * _al(n * ld * 4) + _al(n16 * ld * jb) + 4 * _al(ld * 4) + _al(ld) + 3 * _al(P * ld * 4)
                + 2 * _al((ld // 32) * 16 * (1 if P <= 16 else 2 if P <= 32 else 4) * 4)
                + _al(P * n) + _al(P * n * 8) + _al((5 * ld + 192) * 4) + _al(m * n * 4) + _al(m * 4))
        assert lib.l0cim_server_request_bytes(m, n, ctypes.byref(sp)) == want
    sp = L.solve_params()
    assert lib.l0cim_server_request_bytes(0, 10, ctypes.byref(sp)) == 0
    assert lib.l0cim_server_arena_overhead(16, 8192, ctypes.byref(sp)) > 16 * ctypes.sizeof(L.Stats)


def test_server_create_rejects_bad_arguments_on_host():
    lib = L.lib()
    cim, sp = L.cim_params(), L.solve_params(replicas=8)
    h = ctypes.c_void_p()
    big = 1 << 30

    def create(c=cim, s=sp, slots=4, max_n=1000, arena=FAKE, nbytes=big):
        return lib.l0cim_server_create(ctypes.byref(c), ctypes.byref(s), slots, max_n, arena, nbytes, None,
                                       ctypes.byref(h))

    assert create(arena=None) == 1
    assert create(slots=0) == 1
    assert create(max_n=20000) == 2
    assert create(s=L.solve_params(replicas=65)) == 1
    assert create(s=L.solve_params(cdp=L.CDP_CHOL_F64)) == 5
    assert create(s=L.solve_params(j_dtype=L.F64)) == 5
    assert create(c=L.cim_params(dt=0.0)) == 1
    assert create(arena=ctypes.c_void_p(0x1004)) == 1          # not 256-byte aligned
    assert create(nbytes=1024) == 3
    assert "arena" in _err(lib)
    assert lib.l0cim_server_step(None, None) == 1
    assert lib.l0cim_server_set_step_budget(None, 0) == 1
    assert lib.l0cim_server_submit(None, 1, 1, FAKE, 1, FAKE, 0, 0, FAKE, FAKE, FAKE) == 1


def test_matrix_tile_pin_roundtrip_on_host():
    assert L.l0cim_matrix_tile_get(3000, 64, L.BF16, "BN") == 0
    L.l0cim_matrix_tile_set(3000, 64, L.BF16, "BN", 32)
    assert L.l0cim_matrix_tile_get(3000, 64, L.BF16, "BN") == 32
    assert L.l0cim_matrix_tile_get(3000, 64, L.FP8E4M3, "BN") == 0
    with pytest.raises(L.L0cimError):
        L.l0cim_matrix_tile_set(3000, 64, L.BF16, "BN", 128)    # 8 x 4 blocks exceed the LDS sums
    with pytest.raises(L.L0cimError):
        L.l0cim_matrix_tile_set(3000, 8, L.F32, "CN", 24)
    L.l0cim_matrix_tile_set(3000, 64, L.BF16, "BN", 0)
    assert L.l0cim_matrix_tile_get(3000, 64, L.BF16, "BN") == 0
