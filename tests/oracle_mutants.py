"""Copies of the oracle's C sources with one planted mistake, compiled like the
oracle itself, so that a test can show that its pins catch the mistake.

Only the copy is edited (in a temporary directory); the oracle's own sources
are never touched.  Each edit must match exactly once, so a planted mistake
cannot silently miss its target when the oracle changes.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import oracle

_SRC_DIR = os.path.dirname(os.path.abspath(oracle.__file__))
_SOURCES = ("p3t_oracle.c", "hard_oracle.c")


def build_mutant(workdir: str, edits) -> str:
    """edits: [(source file name, exact text, replacement)]; returns the .so path."""
    os.makedirs(workdir, exist_ok=True)
    for f in _SOURCES:
        shutil.copy(os.path.join(_SRC_DIR, f), os.path.join(workdir, f))
    for fname, old, new in edits:
        path = os.path.join(workdir, fname)
        text = open(path).read()
        count = text.count(old)
        if count != 1:
            raise AssertionError(f"planted edit matches {count} times in {fname}: {old!r}")
        open(path, "w").write(text.replace(old, new))
    lib = os.path.join(workdir, "liboracle_mutant.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, *[os.path.join(workdir, f) for f in _SOURCES],
                           "-o", lib, "-lm"])
    return lib
