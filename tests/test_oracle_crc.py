"""Pins for the oracle's CRC-32C: published vectors, an independent hardware
implementation, the bitwise definition, and the linearity of CRCs over GF(2)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


def _parse_input(spec: str) -> bytes:
    spec = spec.strip()
    if spec == "empty":
        return b""
    kind, _, rest = spec.partition(":")
    if kind == "ascii":
        return rest.encode("ascii")
    if kind == "repeat":
        b, n = rest.split(":")
        return bytes([int(b, 16)]) * int(n)
    if kind == "range":
        a, b = (int(x, 16) for x in rest.split(":"))
        step = 1 if b >= a else -1
        return bytes(range(a, b + step, step))
    raise ValueError(spec)


def _vectors():
    out = []
    with open(os.path.join(HERE, "golden", "crc32c_vectors.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, inp, exp = (x.strip() for x in line.split("|"))
            out.append((name, _parse_input(inp), int(exp, 16)))
    return out


@pytest.fixture(scope="module")
def hw_crc(tmp_path_factory):
    d = tmp_path_factory.mktemp("hwcrc")
    so = str(d / "libhwcrc.so")
    subprocess.run(["gcc", "-O2", "-msse4.2", "-fPIC", "-shared", "-o", so,
                    os.path.join(HERE, "crc32c_sse42.c")], check=True)
    L = ctypes.CDLL(so)
    L.hw_crc32c.restype = ctypes.c_uint32
    L.hw_crc32c.argtypes = [ctypes.c_char_p, ctypes.c_uint64]
    return lambda b: L.hw_crc32c(bytes(b), len(b))


@pytest.mark.parametrize("name,data,expected", _vectors())
def test_published_vectors(name, data, expected, hw_crc):
    assert oracle.crc32c(data) == expected, name
    assert brute.crc32c_bitwise(data) == expected, name
    assert hw_crc(data) == expected, name


def test_table_equals_bitwise_and_hardware(hw_crc):
    rng = np.random.default_rng(11)
    for n in list(range(0, 70)) + [255, 256, 257, 1000, 4096]:
        data = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        c = oracle.crc32c(data)
        assert c == brute.crc32c_bitwise(data)
        assert c == hw_crc(data)


def test_hardware_on_large_pages(hw_crc):
    rng = np.random.default_rng(12)
    for n in [4096, 65536, 2 << 20]:
        data = rng.integers(0, 256, n, dtype=np.uint8)
        assert oracle.crc32c(data) == hw_crc(data.tobytes())


def test_affine_xor_property():
    # CRC-32C is affine over GF(2): for equal-length messages the constant
    # terms cancel in an odd-sized XOR, so crc(A)^crc(B)^crc(C) == crc(A^B^C).
    rng = np.random.default_rng(13)
    for n in [1, 7, 64, 4096]:
        a, b, c = (rng.integers(0, 256, n, dtype=np.uint8) for _ in range(3))
        lhs = oracle.crc32c(a) ^ oracle.crc32c(b) ^ oracle.crc32c(c)
        assert lhs == oracle.crc32c(a ^ b ^ c)


def test_single_bit_errors_change_crc():
    rng = np.random.default_rng(14)
    data = rng.integers(0, 256, 512, dtype=np.uint8)
    c0 = oracle.crc32c(data)
    for bit in range(0, 512 * 8, 37):
        d = data.copy()
        d[bit // 8] ^= np.uint8(1 << (bit % 8))
        assert oracle.crc32c(d) != c0
