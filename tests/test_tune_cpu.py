"""Host logic of the autotuner cache (include/spkadd_tune.h): shape-class keys, store
and lookup, the JSON file round trip and its validation.  No device is needed."""
import json
import os

import pytest

ARCH = "gfx950:sramecc+:xnack-"


@pytest.fixture()
def B():
    from paper_2112_10223_amd import binding
    binding.tune_clear()
    yield binding
    binding.tune_clear()


def test_key_classes(B):
    k = B.tune_key(65536, 65536, 32, 65536 * 512, arch=ARCH, cus=256)
    assert (k.m_log2, k.n_log2, k.k_log2, k.u_log2) == (16, 16, 5, 9)
    k = B.tune_key(65537, 1, 1, 0, arch=ARCH, cus=256)
    assert (k.m_log2, k.n_log2, k.k_log2, k.u_log2) == (17, 0, 0, 0)
    k = B.tune_key(3, 10, 3, 31, arch=ARCH, cus=256)  # mean u = ceil(31 / 10) = 4
    assert (k.m_log2, k.n_log2, k.k_log2, k.u_log2) == (2, 4, 2, 2)


def test_store_lookup_keeps_other_fields(B):
    k = B.tune_key(4096, 4096, 8, 4096 * 100, arch=ARCH, cus=256)
    assert B.tune_lookup(k) is None
    B.tune_store(k, B.make_opts(wave_max=512, accum_mode=1, bitmap_ratio=2.0, wave_merge=1, window_cap=4096,
                                load_factor_sym=0.35, window_fill=0.5), 1.25)
    base = B.make_opts(flags=1, force_bin=3, hash_mode=1, wave_max=1024)
    got = B.tune_lookup(k, base)
    assert (got.wave_max, got.accum_mode, got.bitmap_ratio, got.wave_merge, got.window_cap) == (512, 1, 2.0, 1, 4096)
    assert abs(got.load_factor_sym - 0.35) < 1e-7 and got.window_fill == 0.5
    assert (got.flags, got.force_bin, got.hash_mode) == (1, 3, 1)  # not tuned: kept
    assert base.wave_max == 1024  # the argument is not modified
    other = B.tune_key(4096, 4096, 8, 4096 * 100, arch=ARCH, cus=128)  # another device class
    assert B.tune_lookup(other) is None


def test_save_load_round_trip(B, tmp_path):
    keys = [B.tune_key(2 ** e, 2 ** e, 4, 2 ** e * 10, dtype=e % 2, arch=ARCH, cus=256) for e in range(4, 10)]
    for i, k in enumerate(keys):
        B.tune_store(k, B.make_opts(wave_max=256 * (1 + i % 4), bitmap_ratio=0.5 * (i + 1)), 0.1 * i)
    p = str(tmp_path / "tune.json")
    B.tune_save(p)
    doc = json.load(open(p))
    assert doc["format"] == "spkadd-tune" and doc["version"] == 2 and len(doc["entries"]) == len(keys)
    B.tune_clear()
    assert B.tune_size() == 0
    B.tune_load(p)
    assert B.tune_size() == len(keys)
    for i, k in enumerate(keys):
        got = B.tune_lookup(k)
        assert got.wave_max == 256 * (1 + i % 4) and got.bitmap_ratio == 0.5 * (i + 1)
    # entries of a loaded file replace those with the same key
    B.tune_store(keys[0], B.make_opts(wave_max=768), 9.0)
    B.tune_load(p)
    assert B.tune_lookup(keys[0]).wave_max == 256


@pytest.mark.parametrize("text", [
    "", "not json", "[]", '{"format": "other", "version": 1, "entries": []}',
    '{"format": "spkadd-tune", "version": 3, "entries": []}',
    '{"format": "spkadd-tune", "version": 1, "entries": [{"arch": "x"}]}',
    '{"format": "spkadd-tune", "version": 1, "entries": [{"arch": "x", "cus": 1, "dtype": 0, "m_log2": 1, '
    '"n_log2": 1, "k_log2": 1, "u_log2": 1, "wave_max": 2000, "accum_mode": 0, "bitmap_ratio": 1, "wave_merge": 0, '
    '"window_cap": 0, "load_factor_sym": 0, "load_factor_num": 0, "window_fill": 0, "ms": 1}]}',
    '{"format": "spkadd-tune", "version": 1, "entries": [', '{"format": "spkadd-tune", "version": 1} extra'])
def test_load_rejects_malformed(B, tmp_path, text):
    k = B.tune_key(100, 100, 2, 100, arch=ARCH, cus=256)
    B.tune_store(k, B.make_opts(wave_max=512))
    p = tmp_path / "bad.json"
    p.write_text(text)
    with pytest.raises(B.SpkaddError) as e:
        B.tune_load(str(p))
    assert e.value.status == B.SPKADD_ERR_INVALID
    assert B.tune_size() == 1 and B.tune_lookup(k).wave_max == 512  # nothing merged


def test_load_save_errors(B, tmp_path):
    with pytest.raises(B.SpkaddError) as e:
        B.tune_load(str(tmp_path / "missing.json"))
    assert e.value.status == B.SPKADD_ERR_STATE
    with pytest.raises(B.SpkaddError) as e:
        B.tune_save(str(tmp_path / "no_dir" / "x.json"))
    assert e.value.status == B.SPKADD_ERR_STATE


V1_ENTRY = ('{"arch": "%s", "cus": 256, "dtype": 0, "m_log2": 12, "n_log2": 12, "k_log2": 3, "u_log2": 7, '
            '"wave_max": 768, "accum_mode": 0, "bitmap_ratio": 2, "wave_merge": 1, "window_cap": 0, '
            '"load_factor_sym": 0.35, "load_factor_num": 0, "window_fill": 0, "ms": 1.5}' % ARCH)


def test_version_1_file_still_loads(B, tmp_path):
    """A file of the first format (no key kind, no batch fields) loads as one-SpKAdd entries."""
    p = tmp_path / "v1.json"
    p.write_text('{"format": "spkadd-tune", "version": 1, "entries": [%s]}' % V1_ENTRY)
    B.tune_load(str(p))
    k = B.tune_key(4096, 4096, 8, 4096 * 100, arch=ARCH, cus=256)
    got = B.tune_lookup(k)
    assert got is not None and got.wave_max == 768 and got.wave_merge == 1 and got.bitmap_ratio == 2.0


def test_batch_entries(B, tmp_path):
    """Batched-path entries (key kind 1) keep their own fields apart from one-SpKAdd
    entries of the same shape class, survive the file round trip, and set only the
    accumulator and batch fields on lookup."""
    plain = B.tune_key(4096, 4096, 8, 4096 * 100, arch=ARCH, cus=256)
    batch = B.tune_key(4096, 4096, 8, 4096 * 100, arch=ARCH, cus=256)
    batch.kind = 1
    B.tune_store(plain, B.make_opts(wave_max=512, bitmap_ratio=4.0), 1.0)
    B.tune_store(batch, B.make_opts(accum_mode=1, batch_fused_cols=-1, batch_wave_max=768, batch_wg_max=3072,
                                    batch_wg_threads=512, batch_run_size=32, wave_max=256), 2.0)
    assert B.tune_size() == 2
    p = str(tmp_path / "t.json")
    B.tune_save(p)
    B.tune_clear()
    B.tune_load(p)
    base = B.make_opts(wave_max=1000, window_cap=2048)
    got = B.tune_lookup(batch, base)
    assert (got.accum_mode, got.batch_fused_cols, got.batch_wave_max, got.batch_wg_max, got.batch_wg_threads,
            got.batch_run_size) == (1, -1, 768, 3072, 512, 32)
    assert got.wave_max == 1000 and got.window_cap == 2048  # one-SpKAdd fields untouched
    got = B.tune_lookup(plain, B.make_opts(batch_run_size=16))
    assert got.wave_max == 512 and got.bitmap_ratio == 4.0 and got.batch_run_size == 16
    bad = json.load(open(p))
    bad["entries"][0]["batch_wg_max"] = 5000
    open(p, "w").write(json.dumps(bad))
    with pytest.raises(B.SpkaddError):
        B.tune_load(p)
