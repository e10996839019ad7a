"""Helpers for the GPU parity tests: device buffers, the library handles, and
the oracle-side rounding of stored operands (FP32, FP16, BF16 round to nearest
even, written from the IEEE-754 definitions; FP16 and BF16 are reached through
FP32 exactly as the library stores them)."""
import numpy as np
import torch

from paper_1811_00355_amd import binding as B


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


def round_f32(z):
    z = np.asarray(z)
    if np.iscomplexobj(z):
        return z.real.astype(np.float32).astype(np.float64) + 1j * z.imag.astype(np.float32).astype(np.float64)
    return z.astype(np.float32).astype(np.float64)


def bf16_bits(x):
    """bfloat16 bit patterns (uint32) of float32 values, round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint32)


def _bf16_real(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_store(z, dtype):
    """Value of z after storage in `dtype` (dd dtype code)."""
    z = np.asarray(z)
    if dtype == B.DD_F64:
        return z.astype(np.complex128) if np.iscomplexobj(z) else z.astype(np.float64)
    if dtype == B.DD_F32:
        return round_f32(z)
    f = (lambda r: np.asarray(r, dtype=np.float32).astype(np.float16).astype(np.float64)) if dtype == B.DD_F16 \
        else _bf16_real
    if np.iscomplexobj(z):
        return f(z.real.astype(np.float32)) + 1j * f(z.imag.astype(np.float32))
    return f(np.asarray(z, dtype=np.float32))


def stored_clover_dense(packed, dtype):
    """Dense [V][12][12] clover-like field from the packed [V][2][36] FP64
    export, after rounding every stored real to `dtype` (the oracle's
    unpacking, so the test compares against what the library stores)."""
    from oracle.dirac import unpack_hermitian6, from_chiral_blocks
    p = round_store(packed, dtype)
    return from_chiral_blocks(unpack_hermitian6(p))


def packed_oracle_clover(A):
    from oracle.dirac import chiral_blocks, pack_hermitian6
    return pack_hermitian6(chiral_blocks(A))


def max_rel(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def fine_apply(gauge, dtype, nrhs, psi, fn):
    """Pack canonical host vectors [nrhs][V][4][3], run fn(packed_in, packed_out), unpack."""
    cin = to_dev(psi.reshape(nrhs, -1))
    pin = gauge.new_packed(dtype, nrhs)
    pout = gauge.new_packed(dtype, nrhs)
    gauge.pack(dtype, nrhs, cin, pin)
    fn(pin, pout)
    cout = torch.zeros_like(cin)
    gauge.unpack(dtype, nrhs, pout, cout)
    torch.cuda.synchronize()
    return to_host(cout).reshape(psi.shape)
