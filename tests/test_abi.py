"""The C ABI on the host: the library loads, exports every entry point that
include/li.h declares, and rejects invalid arguments before touching the GPU
(every call here fails validation, so no HIP work is issued)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "li.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(li_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def li():
    from paper_2312_13170_amd import li as mod
    return mod


def test_header_declares_entry_points():
    syms = _declared_symbols()
    for s in ["li_gemm", "li_gemm_ex", "li_mm2", "li_covariance", "li_correlation",
              "li_group_plan_create", "li_group_plan_launch", "li_tune_set", "li_last_error"]:
        assert s in syms


def test_every_declared_symbol_is_exported(li):
    lib = ctypes.CDLL(li.LIB_PATH)
    for s in _declared_symbols():
        assert hasattr(lib, s), s
    assert set(_declared_symbols()) == set(li.EXPORTED)


def test_version(li):
    assert "gfx950" in li.li_version()


FAKE = 1 << 40  # a host integer used as a device address; never dereferenced


def _status(li, fn, *args):
    return fn(*args)


def test_negative_sizes_rejected(li):
    lib = li._lib
    assert lib.li_gemm(-1, 4, 4, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, None) == li.LI_ERR_INVALID_SIZE
    assert "M" in li.li_last_error()
    assert lib.li_mm2(4, -2, 4, 4, 1.0, 0.0, FAKE, FAKE, FAKE, FAKE, FAKE, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_covariance(-3, 8, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == li.LI_ERR_INVALID_SIZE


def test_null_pointers_rejected(li):
    lib = li._lib
    assert lib.li_gemm(4, 4, 4, 1.0, None, FAKE, 0.0, FAKE + 4096, None) == li.LI_ERR_NULL_POINTER
    assert lib.li_gemm(4, 4, 4, 1.0, FAKE, FAKE + 4096, 0.0, None, None) == li.LI_ERR_NULL_POINTER
    assert "C" in li.li_last_error()


def test_overlap_rejected(li):
    lib = li._lib
    # C (64x64 floats) starts inside A
    assert lib.li_gemm(64, 64, 64, 1.0, FAKE, FAKE + (1 << 20), 0.0, FAKE + 100, None) == li.LI_ERR_OVERLAP
    # mm2: D overlapping tmp
    n = 16
    b = 4 * n * n
    st = lib.li_mm2(n, n, n, n, 1.0, 1.0, FAKE, FAKE + b, FAKE + 2 * b, FAKE + 3 * b, FAKE + 2 * b + 8, None)
    assert st == li.LI_ERR_OVERLAP


def test_covariance_argument_rules(li):
    lib = li._lib
    M, N = 8, 16
    xb = 4 * M * N
    ws = lib.li_stats_workspace_bytes(M, N)
    assert ws > 0
    # N < 2 is undefined for the unbiased covariance
    assert lib.li_covariance(M, 1, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 3 * xb, FAKE + 4 * xb, ws, None) == li.LI_ERR_INVALID_SIZE
    # workspace too small
    assert lib.li_covariance(M, N, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 3 * xb, FAKE + 4 * xb, ws - 8, None) == li.LI_ERR_WORKSPACE
    # data_out partially overlapping data
    assert lib.li_covariance(M, N, FAKE, FAKE + 4, FAKE + 2 * xb, FAKE + 3 * xb, FAKE + 4 * xb, ws, None) == li.LI_ERR_OVERLAP
    # mean overlapping cov
    assert lib.li_covariance(M, N, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 2 * xb + 8, FAKE + 4 * xb, ws, None) == li.LI_ERR_OVERLAP
    # correlation: negative eps
    assert lib.li_correlation(M, N, -0.1, FAKE, FAKE, FAKE + 2 * xb, FAKE + 3 * xb, FAKE + 4 * xb,
                              FAKE + 8 * xb, ws, None) == li.LI_ERR_INVALID_SIZE


def test_rank_update_argument_rules(li):
    lib = li._lib
    N, K = 16, 8
    ab, cb = 4 * N * K, 4 * N * N
    ws = lib.li_syrk_workspace_bytes(N, K)
    assert ws > 0 and lib.li_syrk_workspace_bytes(0, K) == 0
    W = FAKE + (1 << 24)
    assert lib.li_syrk(-1, K, 1.0, FAKE, 0.0, FAKE + ab, W, ws, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_syrk(N, K, 1.0, None, 0.0, FAKE + ab, W, ws, None) == li.LI_ERR_NULL_POINTER
    # C inside A
    assert lib.li_syrk(N, K, 1.0, FAKE, 0.0, FAKE + 4, W, ws, None) == li.LI_ERR_OVERLAP
    # workspace too small, and overlapping C
    assert lib.li_syrk(N, K, 1.0, FAKE, 0.0, FAKE + ab, W, ws - 4, None) == li.LI_ERR_WORKSPACE
    assert lib.li_syrk(N, K, 1.0, FAKE, 0.0, FAKE + ab, FAKE + ab + 16, ws, None) == li.LI_ERR_OVERLAP
    # syr2k: B NULL, C overlapping B
    assert lib.li_syr2k(N, K, 1.0, FAKE, None, 0.0, FAKE + 2 * ab, W, ws, None) == li.LI_ERR_NULL_POINTER
    assert lib.li_syr2k(N, K, 1.0, FAKE, FAKE + ab, 0.0, FAKE + ab + 4, W, ws, None) == li.LI_ERR_OVERLAP
    # alpha == 0: operands are not read, so NULL A / B and no workspace pass
    # validation (the call then needs the device, absent here)
    st = lib.li_syr2k(N, K, 0.0, None, None, 1.0, FAKE + cb, None, 0, None)
    assert st in (li.LI_OK, li.LI_ERR_UNSUPPORTED_DEVICE)


def test_mm3_argument_rules(li):
    lib = li._lib
    n = 16
    b = 4 * n * n
    A, B, C, D, E, F, G = (FAKE + i * b for i in range(7))
    assert lib.li_mm3(n, n, n, n, -1, A, B, C, D, E, F, G, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_mm3(n, n, n, n, n, A, B, C, D, None, F, G, None) == li.LI_ERR_NULL_POINTER
    # G overlapping F, E overlapping D
    assert lib.li_mm3(n, n, n, n, n, A, B, C, D, E, F, F + 4, None) == li.LI_ERR_OVERLAP
    assert lib.li_mm3(n, n, n, n, n, A, B, C, D, D + 8, F, G, None) == li.LI_ERR_OVERLAP


def test_gemm_form_validation(li):
    lib = li._lib
    assert lib.li_gemm_form(5, 8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, None) == li.LI_ERR_BAD_ENUM
    assert lib.li_gemm_form(0, -8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_gemm_form(1, 8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 16, None) == li.LI_ERR_OVERLAP
    assert lib.li_gemm_form(2, 2000000, 8, 8, 1.0, FAKE, FAKE + (1 << 30), 0.0, FAKE + (1 << 31), None) == li.LI_ERR_INVALID_SIZE


def test_precision_enum_and_workspace(li):
    lib = li._lib
    assert lib.li_gemm_ex(8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, 9, None, 0, None) == li.LI_ERR_BAD_ENUM
    need = lib.li_gemm_ex_workspace_bytes(8, 8, 8, li.LI_BF16X3)
    assert need >= 2 * 2 * 8 * 8
    assert lib.li_gemm_ex(8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, li.LI_BF16X3, FAKE + (1 << 20), need - 2, None) == li.LI_ERR_WORKSPACE
    assert lib.li_round16(16, FAKE, FAKE + 64, FAKE + 128, li.LI_FP16, None) == li.LI_ERR_BAD_ENUM


def test_tuning_table(li):
    for k in (li.LI_KERNEL_GEMM_F32, li.LI_KERNEL_SYRK_F32, li.LI_KERNEL_GEMM_LP,
              li.LI_KERNEL_SYRK_ROWS, li.LI_KERNEL_GEMM_LP_SPLIT):
        n = li.li_tune_num_candidates(k)
        assert n >= 3
        for i in range(n):
            c = li.li_tune_candidate(k, i)
            assert c["bm"] % 32 == 0 and c["bn"] % 32 == 0 and c["bk"] % 8 == 0
            if k in (li.LI_KERNEL_SYRK_F32, li.LI_KERNEL_SYRK_ROWS):
                assert c["bm"] == c["bn"]
    assert li.li_tune_bucket(2048, 2048, 2048) == 12
    assert li.li_tune_bucket(1, 1, 1) == 1
    b = li.li_tune_bucket(300, 200, 100)
    old = li.li_tune_get(li.LI_KERNEL_GEMM_F32, b)
    try:
        li.li_tune_set(li.LI_KERNEL_GEMM_F32, b, 3)
        assert li.li_tune_get(li.LI_KERNEL_GEMM_F32, b) == 3
        li.li_tune_set(li.LI_KERNEL_GEMM_F32, b, -1)
        assert li.li_tune_get(li.LI_KERNEL_GEMM_F32, b) == -1
        with pytest.raises(li.LiError):
            li.li_tune_set(li.LI_KERNEL_GEMM_F32, b, 999)
    finally:
        li.li_tune_set(li.LI_KERNEL_GEMM_F32, b, old)
    with pytest.raises(li.LiError):
        li.li_tune_force(7, 0)
    assert li.li_tune_pick(7, 8, 8, 8) == -1 and li.li_tune_pick(li.LI_KERNEL_GEMM_F32, -1, 8, 8) == -1


def test_tile_choice_by_output_size(li):
    # The GEMM and row-form families choose by the output's size (a long
    # reduction does not take the tile of a larger square problem); the
    # covariance family by its order and the class of the sample count.
    F, S, R = li.LI_KERNEL_GEMM_F32, li.LI_KERNEL_SYRK_F32, li.LI_KERNEL_SYRK_ROWS
    b12, b13 = li.li_tune_bucket(2048, 2048, 0), li.li_tune_bucket(4096, 4096, 4096)
    assert (b12, b13) == (12, 13)
    for k in (F, li.LI_KERNEL_GEMM_LP, li.LI_KERNEL_GEMM_LP_SPLIT):
        assert li.li_tune_key(k, 2048, 2048, 4096) == 12
        assert li.li_tune_key(k, 8192, 512, 64) == 12
        assert li.li_tune_key(k, 8192, 2048, 64) == 13
    # covariance: order bits + 16 * sample class (N / M: <1.5, <3, <6, more)
    for n, slot in ((2048, 12), (3071, 12), (3072, 28), (4096, 28), (6143, 28), (6144, 44),
                    (12287, 44), (12288, 60), (1, 12), (0, 12)):
        assert li.li_tune_key(S, 2048, 2048, n) == slot, n
    assert li.li_tune_key(S, 65536, 65536, 65536) == 15
    # row-form updates: order bits + 16 * rank class (K / N: <0.75, <3, <12, more)
    for k, slot in ((511, 12), (1535, 12), (1536, 28), (2048, 28), (6143, 28), (6144, 44),
                    (24575, 44), (24576, 60), (65536, 60)):
        assert li.li_tune_key(R, 2048, 2048, k) == slot, k
    assert li.li_tune_key(S, 0, 0, 5) == 48
    assert li.li_tune_key(li.LI_KERNEL_GROUPED_COV, 300, 300, 5000) == 13
    assert li.li_tune_key(7, 8, 8, 8) == -1 and li.li_tune_key(S, 8, 8, -1) == -1
    old = {(k, b): li.li_tune_get(k, b) for k in (F, S, R) for b in (b12, b13, 28, 30, 6, 14, 46, 62)}
    try:
        # slots without an entry: stream-K for a large result or a long
        # reduction, 64 x 64 tiles for a short one over a small result
        for b in (30, 6):
            li.li_tune_set(S, b, -1)
        assert li.li_tune_pick(S, 8192, 8192, 16384) == 20
        assert li.li_tune_key(S, 40, 40, 50) == 6 and li.li_tune_pick(S, 40, 40, 50) == 17
        for b in (14, 30, 46, 62):  # 8192 at every rank class
            li.li_tune_set(R, b, -1)
        assert li.li_tune_pick(R, 8192, 8192, 1024) == 10
        assert li.li_tune_pick(R, 8192, 8192, 8192) == 15
        assert li.li_tune_pick(R, 8192, 8192, 131072) == 15
        for k in (F, S, R):
            li.li_tune_set(k, b12, 1)
            li.li_tune_set(k, b13, 2)
        li.li_tune_set(S, 28, 3)
        assert li.li_tune_pick(F, 2048, 2048, 4096) == 1
        assert li.li_tune_pick(F, 2048, 2048, 1024) == 1
        assert li.li_tune_pick(F, 4096, 4096, 256) == 2
        # by area: 8192 x 512 is the square of side 2048
        assert li.li_tune_pick(F, 8192, 512, 8192) == 1
        assert li.li_tune_pick(F, 512, 8192, 8192) == 1
        assert li.li_tune_pick(F, 8192, 2048, 64) == 2
        assert li.li_tune_pick(R, 2048, 2048, 500) == 1
        assert li.li_tune_pick(S, 2048, 2048, 4096) == 3
        assert li.li_tune_pick(S, 2048, 2048, 2048) == 1
        assert li.li_tune_pick(S, 4096, 4096, 4096) == 2
        li.li_tune_force(F, 0)
        assert li.li_tune_pick(F, 2048, 2048, 4096) == 0
    finally:
        li.li_tune_force(F, -1)
        for (k, b), v in old.items():
            li.li_tune_set(k, b, v)
    # the grouped families list the plans' shape classes (square tiles)
    for k in (li.LI_KERNEL_GROUPED_GEMM, li.LI_KERNEL_GROUPED_COV):
        n = li.li_tune_num_candidates(k)
        assert n >= 2
        for i in range(n):
            c = li.li_tune_candidate(k, i)
            assert c["bm"] == c["bn"] and c["split_k"] == 1
        with pytest.raises(li.LiError):
            li.li_tune_force(k, n)


def test_wave_quantisation(li):
    # The table's FP32 GEMM choices are searched on square powers of two;
    # other sizes of a slot take the steady tile shape with the fewest
    # wasted tile slots in the last round (256 compute units), when the
    # table's shape is predicted more than 5% slower.
    F = li.LI_KERNEL_GEMM_F32
    slots = {11: 20, 12: 44, 13: 49}
    old = {b: li.li_tune_get(F, b) for b in slots}
    try:
        for b, c in slots.items():
            li.li_tune_set(F, b, c)
        # the searched squares keep their entries
        assert li.li_tune_pick(F, 2048, 2048, 2048) == 44
        assert li.li_tune_pick(F, 4096, 4096, 4096) == 49
        assert li.li_tune_pick(F, 1024, 1024, 1024) == 20   # below 1536^2: the table stands
        # 3072^2 in 128 x 128 tiles: 576 tiles, 3 rounds for 2.25; 64 x 64: 2304, 9 rounds
        assert li.li_tune_pick(F, 3072, 3072, 3072) == 19
        # 4500^2: 648 tiles of 128 x 256 (3 rounds for 2.53); 64 x 128: 2556 (10 for 9.98)
        assert li.li_tune_pick(F, 4500, 4500, 4500) == 25
        # 6144^2: 1152 tiles of 128 x 256 (5 for 4.5); 128 x 128: 2304 (9 exactly)
        assert li.li_tune_pick(F, 6144, 6144, 2048) == 44
        assert li.li_tune_pick(F, 1536, 1536, 1536) == 19
        # within 5% of the best: 8192 x 1024 stays on the slot's 128 x 128
        assert li.li_tune_pick(F, 8192, 1024, 4096) == 44
        li.li_tune_force(F, 49)
        assert li.li_tune_pick(F, 3072, 3072, 3072) == 49
    finally:
        li.li_tune_force(F, -1)
        for b, v in old.items():
            li.li_tune_set(F, b, v)
    # bf16 / fp16: 128 x 128 tiles (candidate 9) up to two rounds, then one
    # round of 256 x 256 tiles (19); split-bf16 alike with its own shapes
    L, LS = li.LI_KERNEL_GEMM_LP, li.LI_KERNEL_GEMM_LP_SPLIT
    old = {(k, b): li.li_tune_get(k, b) for k in (L, LS) for b in (12, 13)}
    try:
        li.li_tune_set(L, 12, 9)
        li.li_tune_set(L, 13, 19)
        li.li_tune_set(LS, 12, 9)
        li.li_tune_set(LS, 13, 16)
        for n, c in ((2048, 9), (2560, 9), (2816, 9), (3072, 19), (3840, 19), (4096, 19), (7000, 19)):
            assert li.li_tune_pick(L, n, n, n) == c, n
        assert li.li_tune_pick(L, 8192, 1024, 8192) == 9
        for n, c in ((2048, 9), (2560, 9), (3072, 16), (3584, 16), (5000, 16)):
            assert li.li_tune_pick(LS, n, n, n) == c, n
    finally:
        for (k, b), v in old.items():
            li.li_tune_set(k, b, v)


def test_split_spill_takes_stream_k(li):
    # A covariance split reduction whose (upper tiles) x (chunks) work-groups
    # spill past one round of 256 compute units with short chunks takes the
    # stream-K schedule of the same tile; long chunks keep the split, and the
    # row-form updates keep their table entries.
    S, R = li.LI_KERNEL_SYRK_F32, li.LI_KERNEL_SYRK_ROWS
    entries = {(S, 27): 10, (S, 59): 10, (R, 26): 9}
    old = {kb: li.li_tune_get(*kb) for kb in entries}
    try:
        for (k, b), c in entries.items():
            li.li_tune_set(k, b, c)
        assert li.li_tune_candidate(S, 10)["split_k"] == 7
        assert li.li_tune_pick(S, 1024, 1024, 2048) == 10    # 36 tiles x 7 = 252
        assert li.li_tune_pick(S, 1500, 1500, 3000) == 20    # 78 x 7 = 546, chunks of 428
        assert li.li_tune_key(S, 1900, 1900, 30000) == 59
        assert li.li_tune_pick(S, 1900, 1900, 30000) == 10   # 120 x 7 = 840, chunks of 4285
        assert li.li_tune_pick(R, 1000, 1000, 2000) == 9     # row form: the table stands
        assert li.li_tune_candidate(S, 20)["split_k"] == 0
    finally:
        for (k, b), v in old.items():
            li.li_tune_set(k, b, v)


def test_group_plan_validation(li):
    P = li.make_problem
    G, COV = li.LI_PROBLEM_GEMM, li.LI_PROBLEM_COVARIANCE
    mb = 4 * 64 * 64
    ok_a = P(G, 64, 64, 64, 1.0, 0.0, FAKE, FAKE + mb, FAKE + 2 * mb)
    # second problem writes into the first one's C
    clash = P(G, 64, 64, 64, 1.0, 0.0, FAKE + 3 * mb, FAKE + 4 * mb, FAKE + 2 * mb + 64)
    with pytest.raises(li.LiError) as e:
        li.li_group_plan_create([ok_a, clash])
    assert e.value.status == li.LI_ERR_OVERLAP
    # an output overlapping another problem's input
    clash2 = P(G, 64, 64, 64, 1.0, 0.0, FAKE + 3 * mb, FAKE + 4 * mb, FAKE + 8)
    with pytest.raises(li.LiError) as e:
        li.li_group_plan_create([ok_a, clash2])
    assert e.value.status == li.LI_ERR_OVERLAP
    with pytest.raises(li.LiError) as e:
        li.li_group_plan_create([P(7, 4, 4, 4, 1.0, 0.0, FAKE, FAKE, FAKE)])
    assert e.value.status == li.LI_ERR_BAD_ENUM
    with pytest.raises(li.LiError) as e:
        li.li_group_plan_create([P(G, 4, 4, 4, 1.0, 0.0, None, FAKE, FAKE + 4096)])
    assert e.value.status == li.LI_ERR_NULL_POINTER
    with pytest.raises(li.LiError) as e:
        li.li_group_plan_create([P(COV, 8, 1, 0, 1.0, 0.0, FAKE, None, FAKE + 4096, FAKE + 8192, FAKE + 16384)])
    assert e.value.status == li.LI_ERR_INVALID_SIZE


def test_tune_table_save_load(li, tmp_path):
    k = li.LI_KERNEL_SYRK_F32
    b1, b2 = 20, 21
    old1, old2 = li.li_tune_get(k, b1), li.li_tune_get(k, b2)
    try:
        li.li_tune_set(k, b1, 1)
        li.li_tune_set(k, b2, 2)
        path = tmp_path / "t.txt"
        li.li_tune_save(str(path))
        text = path.read_text()
        assert "%d %d 1" % (k, b1) in text and "%d %d 2" % (k, b2) in text
        li.li_tune_set(k, b1, -1)
        li.li_tune_set(k, b2, -1)
        li.li_tune_load(str(path))
        assert li.li_tune_get(k, b1) == 1 and li.li_tune_get(k, b2) == 2
        # a malformed file changes nothing
        bad = tmp_path / "bad.txt"
        bad.write_text("%d %d 0\n%d 999 0\n" % (k, b1, k))
        with pytest.raises(li.LiError):
            li.li_tune_load(str(bad))
        assert li.li_tune_get(k, b1) == 1
        with pytest.raises(li.LiError) as e:
            li.li_tune_load(str(tmp_path / "missing.txt"))
        assert e.value.status == li.LI_ERR_NOT_FOUND
    finally:
        li.li_tune_set(k, b1, old1)
        li.li_tune_set(k, b2, old2)


def test_matvec_argument_rules(li):
    lib = li._lib
    M, N = 16, 8
    ab = 4 * M * N
    ws = lib.li_matvec_workspace_bytes(M, N)
    assert ws > 0 and lib.li_matvec_workspace_bytes(0, N) == 0
    W = FAKE + (1 << 24)
    x, t, y = FAKE + ab, FAKE + ab + 4096, FAKE + ab + 8192
    assert lib.li_atax(-1, N, FAKE, x, t, y, W, ws, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_atax(M, N, None, x, t, y, W, ws, None) == li.LI_ERR_NULL_POINTER
    assert lib.li_atax(M, N, FAKE, x, x + 4, y, W, ws, None) == li.LI_ERR_OVERLAP
    assert lib.li_atax(M, N, FAKE, x, t, y, W, ws - 4, None) == li.LI_ERR_WORKSPACE
    assert lib.li_atax(M, N, FAKE, x, t, y, FAKE + 16, ws, None) == li.LI_ERR_OVERLAP
    # mvt: x1 overlapping x2 (both in/out)
    assert lib.li_mvt(M, N, FAKE, x, x + 1024, t, t + 16, W, ws, None) == li.LI_ERR_OVERLAP
    # gesummv: B NULL, y overlapping B
    assert lib.li_gesummv(M, N, 1.0, 1.0, FAKE, None, x, t, y, W, ws, None) == li.LI_ERR_NULL_POINTER
    assert lib.li_gesummv(M, N, 1.0, 1.0, FAKE, FAKE + 2 * ab, x, t, FAKE + 2 * ab + 8, W, ws,
                          None) == li.LI_ERR_OVERLAP
    # bicg: r shorter region overlapping s
    assert lib.li_bicg(M, N, FAKE, x, t, y, t + 8, W, ws, None) == li.LI_ERR_OVERLAP


def test_fused_statistics_argument_rules(li):
    lib = li._lib
    M, N = 8, 16
    xb = 4 * M * N
    ws = lib.li_stats_workspace_bytes(M, N)
    # no data_out: the only outputs are mean, (stddev,) cov / corr
    assert lib.li_covariance_fused(M, 1, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 4 * xb, ws, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_covariance_fused(M, N, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 4 * xb, ws - 8, None) == li.LI_ERR_WORKSPACE
    assert lib.li_covariance_fused(M, N, FAKE, FAKE + 8, FAKE + 2 * xb, FAKE + 4 * xb, ws, None) == li.LI_ERR_OVERLAP
    assert lib.li_correlation_fused(M, N, 0.1, FAKE, FAKE + xb, None, FAKE + 2 * xb, FAKE + 4 * xb, ws,
                                    None) == li.LI_ERR_NULL_POINTER


def test_binding_refuses_to_load_without_library(tmp_path):
    # A copy of the binding in a folder with no libli.so must raise on
    # import: the package has no path that computes without the library.
    import importlib.util
    src = os.path.join(ROOT, "paper_2312_13170_amd", "li.py")
    dst = tmp_path / "li.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("li_without_library", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="no fallback"):
        spec.loader.exec_module(mod)


def test_misaligned_workspace_rejected(li):
    # every workspace must be 16-byte aligned (the kernels access it with
    # 16-byte vectors); an address 8 bytes off is refused before any launch
    lib = li._lib
    M, N = 9, 16
    xb = 4 * M * N
    W = FAKE + (1 << 24)
    ws = lib.li_stats_workspace_bytes(M, N)
    assert lib.li_covariance(M, N, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 3 * xb, W + 8, ws, None) == li.LI_ERR_WORKSPACE
    assert "aligned" in li.li_last_error()
    assert lib.li_covariance_fused(M, N, FAKE, FAKE + 2 * xb, FAKE + 3 * xb, W + 8, ws, None) == li.LI_ERR_WORKSPACE
    n, k = 16, 8
    ab = 4 * n * k
    ws = lib.li_syrk_workspace_bytes(n, k)
    assert lib.li_syrk(n, k, 1.0, FAKE, 0.0, FAKE + ab, W + 4, ws, None) == li.LI_ERR_WORKSPACE
    need = lib.li_gemm_ex_workspace_bytes(8, 8, 8, li.LI_BF16)
    assert lib.li_gemm_ex(8, 8, 8, 1.0, FAKE, FAKE + 4096, 0.0, FAKE + 8192, li.LI_BF16, W + 8, need, None) == li.LI_ERR_WORKSPACE
    ws = lib.li_matvec_workspace_bytes(32, 32)
    assert lib.li_bicg(32, 32, FAKE, FAKE + 8192, FAKE + 8320, FAKE + 8448, FAKE + 8576, W + 12, ws, None) == li.LI_ERR_WORKSPACE



def test_no_alloc_covariance_argument_rules(li):
    # the covariance that allocates nothing validates like li_covariance and
    # refuses, before touching the device, a problem whose partials would not
    # fit its fixed array
    lib = li._lib
    assert li.LI_NOALLOC_SCRATCH_BYTES == 64 << 20
    M, N = 8, 16
    xb = 4 * M * N
    assert lib.li_covariance_noalloc(-1, N, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 3 * xb, None) == li.LI_ERR_INVALID_SIZE
    assert lib.li_covariance_noalloc(M, 1, FAKE, FAKE + xb, FAKE + 2 * xb, FAKE + 3 * xb, None) == li.LI_ERR_INVALID_SIZE
    li.li_tune_force(li.LI_KERNEL_SYRK_F32, 9)  # seven split-k copies of every upper tile
    try:
        G = 1 << 30
        assert lib.li_covariance_noalloc(4096, 64, FAKE, FAKE + G, FAKE + 2 * G, FAKE + 3 * G, None) == li.LI_ERR_WORKSPACE
        assert "scratch" in li.li_last_error()
    finally:
        li.li_tune_force(li.LI_KERNEL_SYRK_F32, -1)
