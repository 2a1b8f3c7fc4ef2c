"""Compile the oracle's C walk simulator (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "walks.c")
LIB = os.path.join(HERE, "liboraclewalks.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB
