"""Compression-kernel choice cache (no GPU): a cached record is returned as
is, with the descriptor's kernel set from it, and without any device call;
records are keyed by shape, precision and chain count."""
import json

import numpy as np


def test_cached_choice_is_used_without_measuring(tmp_path, monkeypatch):
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd import api, autotune

    def no_device(*a, **k):
        raise AssertionError("a cached choice must not be measured again")

    monkeypatch.setattr(api, "peps_autotune_compression", no_device)
    desc = p.Desc(4, 4, 2, 4)
    configs = np.zeros((8, 16), dtype=np.uint8)
    cache = tmp_path / "tune.json"
    key = autotune._key(desc, 8)
    cache.write_text(json.dumps({key: {"best": "lds", "ms": [-1.0, 0.3, 0.1, 0.5]}}))
    tuned, rec = p.tune_compression(desc, None, configs, cache_path=str(cache))
    assert rec["cached"] and rec["best"] == "lds"
    assert tuned.compress_kernel == p.COMPRESS_LDS and desc.compress_kernel == p.COMPRESS_AUTO
    # other precisions or chain counts are other records
    assert autotune._key(p.Desc(4, 4, 2, 4, precision=p.PREC_MIXED), 8) != key
    assert autotune._key(desc, 16) != key
