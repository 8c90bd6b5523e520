"""Host logic of bench.py, without a GPU: it measures one GPU only, and its
algorithmic byte model of the benchmark mesh (256x256x16, FP32, p = 4)
matches the layouts of the buffers each kernel reads and writes."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_bytes_of_the_benchmark_mesh():
    sys.path.insert(0, ROOT)
    import bench
    kb = bench.kernel_bytes((256, 256, 16), 4, 4)
    N = 256 * 256 * 16
    vec = 3 * N * 4                      # one [3][N] FP32 field
    Kx, Py, Pz = 257, 512, 32            # x spectrum columns, padded y and z
    sA = 3 * 16 * 256 * Kx * 8           # x-pass spectrum [3][nz][ny][Kx] complex FP32
    sB = 3 * 16 * Py * Kx * 8            # y-pass spectrum [3][nz][Py][Kx]
    kern = 6 * Kx * (Py // 2 + 1) * (Pz // 2 + 1) * 4  # folded real kernel, 6 components
    assert kb["xfwd"] == vec + sA
    assert kb["yfwd"] == kb["yinv"] == sA + sB
    assert kb["zmul"] == 2 * sB + kern == 128004504
    assert kb["xinv"] == sA + 4 * vec                 # spectrum and M in; F, G, next input out
    assert kb["epoly"] == 7 * vec                     # 5 stored fields in, 2 out
    assert kb["extrap"] == 5 * vec                    # M_k, E, M0 in; F, next input out
    assert kb["final"] == 7 * vec                     # M_k, E, M0, F1..F3 in; M out
