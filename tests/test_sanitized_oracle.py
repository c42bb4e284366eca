"""The oracle's CPU pins under AddressSanitizer and UndefinedBehaviorSanitizer:
oracle/rzo.c built with -fsanitize=address,undefined (no recovery) and every
tests/test_oracle_*.py file run against that build in a child interpreter.
Any out-of-bounds access, use after free or undefined operation (a null
pointer handed to memcpy, a signed overflow, a shift out of range) aborts the
child and fails this test."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_pins_clean_under_asan_and_ubsan():
    from oracle import sanitize

    sanitize.build()
    rc, out = sanitize.run()
    assert rc == 0, out[-4000:]
    assert " passed" in out and "failed" not in out
