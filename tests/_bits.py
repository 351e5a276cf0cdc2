"""Bitmap helpers for the tests (LSB-first within each byte)."""
import numpy as np


def bit(buf, i):
    return (int(buf[i // 8]) >> (i % 8)) & 1


def unpack(buf, n):
    return np.unpackbits(np.asarray(buf, dtype=np.uint8), bitorder="little")[:n]
