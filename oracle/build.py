"""Compile the oracle's C parts (test infrastructure): the walk simulator,
the CSR forward / back-accumulation passes for very large graphs and the
edge counter of Algorithm 3's level rule."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "walks.c")
LIB = os.path.join(HERE, "liboraclewalks.so")
LINEAR_SRC = os.path.join(HERE, "linear.c")
LINEAR_LIB = os.path.join(HERE, "liboraclelinear.so")
LDE_SRC = os.path.join(HERE, "lde_count.c")
LDE_LIB = os.path.join(HERE, "liboraclelde.so")


def _compile(src: str, lib: str, force: bool) -> str:
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", src, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


def build(force: bool = True) -> str:
    _compile(LINEAR_SRC, LINEAR_LIB, force)
    _compile(LDE_SRC, LDE_LIB, force)
    return _compile(SRC, LIB, force)


def build_lde(force: bool = True) -> str:
    return _compile(LDE_SRC, LDE_LIB, force)


def build_linear(force: bool = True) -> str:
    return _compile(LINEAR_SRC, LINEAR_LIB, force)
