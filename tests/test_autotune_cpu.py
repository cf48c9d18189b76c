"""CPU checks of the autotuner's cache key (paper_1111_3297_amd/autotune.py)."""


def test_signature_carries_tuner_version_and_classes():
    from paper_1111_3297_amd import autotune
    s = autotune.signature(20, [(0, 4, 1000), (5, 3, 70000)])
    assert s == "v%d|l=20|nreq=2|bits=2^23|B=2^17" % autotune.TUNER_VERSION
    # entries written by an older candidate set do not match a current key
    old = {"l=20|nreq=2|bits=2^23|B=2^17": {"tile_log2": 20}}
    assert s not in old
