"""Roofline constants measured on the GPU (libprism_mb.so, csrc/microbench.hip).

    python -m paper_2604_00250_amd.microbench     -> one JSON line

fma_lane_ops_per_s  FP32 FMA lane-instructions per second (8 independent chains)
exp_lane_ops_per_s  v_exp_f32 lane-instructions per second
q_exp               issue cost of one exp in FMA slots (fma rate / exp rate)
mix14_overlap       fraction of the exp time hidden when 14 FMAs surround each
                    exp (1 = exps fully overlap the FMAs, 0 = fully serial)
copy_GBps           device-to-device copy bandwidth (read + write bytes / s)
"""
import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libprism_mb.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} missing: run `python -m paper_2604_00250_amd.build`")
        L = ctypes.CDLL(LIB)
        for name in ("mb_fma", "mb_exp", "mb_mix14"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            getattr(L, name).restype = ctypes.c_int
        L.mb_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.mb_copy.restype = ctypes.c_int
        _lib = L
    return _lib


def _time(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return best


def run(blocks=256 * 16, iters=4096):
    import torch
    L = lib()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lanes = blocks * 256 * 8 * iters
    t_fma = _time(lambda: L.mb_fma(ctypes.c_void_p(out.data_ptr()), blocks, iters, s))
    t_exp = _time(lambda: L.mb_exp(ctypes.c_void_p(out.data_ptr()), blocks, iters, s))
    t_mix = _time(lambda: L.mb_mix14(ctypes.c_void_p(out.data_ptr()), blocks, iters, s))
    fma_rate = lanes / t_fma
    exp_rate = lanes / t_exp
    t14 = 14 * lanes / fma_rate
    te = lanes / exp_rate
    overlap = max(0.0, min(1.0, (t14 + te - t_mix) / te))
    n = 1 << 28  # 1 GiB per buffer
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    t_copy = _time(lambda: L.mb_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), n, s))
    res = dict(fma_lane_ops_per_s=fma_rate, exp_lane_ops_per_s=exp_rate, q_exp=fma_rate / exp_rate,
               mix14_overlap=overlap, mix14_s=t_mix, copy_GBps=2 * 4 * n / t_copy / 1e9,
               copy_bytes=2 * 4 * n, blocks=blocks, iters=iters)
    return res


if __name__ == "__main__":
    print(json.dumps(run()))
