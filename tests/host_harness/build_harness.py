"""Compile the host build of the library's coefficient math for CPU tests."""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    src = os.path.join(HERE, "zt_host.cpp")
    inl = os.path.join(HERE, "..", "..", "paper_2303_05006_amd", "csrc", "zt_integrals.inl")
    out = os.path.join(HERE, "libzt_host.so")
    if (not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(src), os.path.getmtime(inl))):
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", out + ".tmp", src])
        os.replace(out + ".tmp", out)
    L = ctypes.CDLL(out)
    P, l, i, d = ctypes.c_void_p, ctypes.c_long, ctypes.c_int, ctypes.c_double
    L.zt_host.argtypes = [P] * 9 + [l, P, P, i, P, P, P]
    L.vinc_host.argtypes = [P] * 9 + [i, P, d, P]
    return L
