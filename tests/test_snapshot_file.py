"""CPU checks of the snapshot file format (nuosc_snapshot_info reads and
checks a file without a device).  Files are built here byte by byte from the
layout the header documents: tag, 64-byte header, FP64 payload, FNV-1a hash."""

import struct

import numpy as np
import pytest

from paper_1907_05560_amd import nuosc


def _fnv1a(data: bytes) -> int:
    h = 14695981039346656037
    for b in data:
        h ^= b
        h = (h * 1099511628211) % (1 << 64)
    return h


def _file(n=3, ne=5, na=4, precision=1, integrator=1, frame=0, last_rejected=1, reserved=0, r=12.5, dr=1e-4,
          acc=7, rej=2, payload=None, nb=None):
    nb = 2 * ne * max(na, 1) if nb is None else nb
    head = struct.pack("<8iqddqq", n, ne, na, precision, integrator, frame, last_rejected, reserved, nb, r, dr,
                       acc, rej)
    assert len(head) == 72
    if payload is None:
        rng = np.random.default_rng(5)
        payload = rng.standard_normal(n * 2 * (2 * ne * max(na, 1)) + max(na, 1) * n).astype("<f8").tobytes()
    body = nuosc.SNAPSHOT_TAG + head + payload
    return body + struct.pack("<Q", _fnv1a(body))


def test_header_is_read_back(tmp_path):
    p = tmp_path / "s.bin"
    p.write_bytes(_file())
    info = nuosc.snapshot_info(str(p))
    assert (info["n_flavors"], info["n_energy"], info["n_angle"]) == (3, 5, 4)
    assert (info["precision"], info["integrator"], info["frame"], info["last_rejected"]) == (1, 1, 0, 1)
    assert info["n_beams"] == 40
    assert (info["r_km"], info["dr_km"]) == (12.5, 1e-4)
    assert (info["accepted"], info["rejected"]) == (7, 2)


def test_single_angle_file(tmp_path):
    p = tmp_path / "s.bin"
    p.write_bytes(_file(n=2, ne=9, na=0))
    info = nuosc.snapshot_info(str(p))
    assert info["n_angle"] == 0 and info["n_beams"] == 18


@pytest.mark.parametrize("damage", ["tag", "flip", "truncate", "nb", "flavors", "flag", "reserved", "missing"])
def test_damaged_files_are_rejected(tmp_path, damage):
    p = tmp_path / "s.bin"
    data = bytearray(_file())
    if damage == "tag":
        data[0:8] = b"NUOSCSN9"
    elif damage == "flip":
        data[100] ^= 0x10            # one payload bit: the hash no longer matches
    elif damage == "truncate":
        data = data[:-9]
    elif damage == "nb":
        data = bytearray(_file(nb=41))
    elif damage == "flavors":
        data = bytearray(_file(n=4))
    elif damage == "flag":
        data = bytearray(_file(last_rejected=2))
    elif damage == "reserved":
        data = bytearray(_file(reserved=5))
    if damage != "missing":
        p.write_bytes(bytes(data))
    with pytest.raises(nuosc.NuoscError) as e:
        nuosc.snapshot_info(str(p))
    assert e.value.status == nuosc.E_INVALID
