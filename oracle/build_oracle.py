"""Compile the oracle's C helpers (oracle/ring.c) with gcc into oracle/_ring.so.

Test infrastructure: the oracle is what the tests check the library against.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ring.c")
OUT = os.path.join(HERE, "_ring.so")


def build(force=True):
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, SRC])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
