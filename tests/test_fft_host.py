"""Host check of the register FFTs of the HIP path (csrc/fft.hpp).

The transforms are __host__ __device__ templates, so they are compiled here
with the host C++ compiler (a stub stands in for the HIP runtime header) and
compared with numpy's FFT on seeded inputs for every line length the
transforms use: prime powers (decimation in time) and coprime products
(prime-factor algorithm), both signs, FP64 and FP32.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIZES = [2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32, 36, 40]

SRC = r"""
#include <cstdio>
#include <cstdlib>
#include "fft.hpp"
using namespace ltmp2;
template <class T, int S, int N> void one(FILE* in, FILE* out) {
  cplx<T> x[N];
  for (int k = 0; k < N; ++k) { double a, b; if (fscanf(in, "%lf %lf", &a, &b) != 2) exit(2); x[k] = {T(a), T(b)}; }
  Fft<T, S, N>::run(x);
  for (int k = 0; k < N; ++k) fprintf(out, "%.17g %.17g\n", double(x[k].x), double(x[k].y));
}
template <class T, int N> void both(FILE* in, FILE* out) { one<T, -1, N>(in, out); one<T, 1, N>(in, out); }
template <class T> void all(FILE* in, FILE* out) {
#define S_(n) both<T, n>(in, out);
  SIZES_
}
int main(int argc, char** argv) {
  FILE* in = fopen(argv[1], "r"); FILE* out = fopen(argv[2], "w");
  all<double>(in, out); all<float>(in, out);
  fclose(in); fclose(out); return 0;
}
"""


@pytest.fixture(scope="module")
def fft_runner(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("ffthost")
    (d / "hip").mkdir()
    (d / "hip" / "hip_runtime.h").write_text(
        "#pragma once\n#define __host__\n#define __device__\n#define __forceinline__ inline\n")
    src = SRC.replace("SIZES_", " ".join(f"S_({n})" for n in SIZES))
    (d / "t.cpp").write_text(src)
    exe = d / "t"
    subprocess.run([gxx, "-std=c++20", "-O1", f"-I{d}",
                    f"-I{os.path.join(ROOT, 'paper_1611_06797_amd', 'csrc')}", "-o", str(exe),
                    str(d / "t.cpp")], check=True, capture_output=True)
    return d, exe


def test_register_ffts_match_numpy(fft_runner):
    d, exe = fft_runner
    rng = np.random.default_rng(11)
    # each precision pass reads the same lines: forward then inverse per size
    lines = []
    for n in SIZES:
        for _ in (0, 1):
            lines.append(rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))
    text = "".join(f"{float(z.real)!r} {float(z.imag)!r}\n" for ln in lines for z in ln)
    (d / "in.txt").write_text(text + text)
    subprocess.run([str(exe), str(d / "in.txt"), str(d / "out.txt")], check=True)
    vals = np.loadtxt(d / "out.txt")
    out = vals[:, 0] + 1j * vals[:, 1]
    pos = 0
    for prec, tol in (("f64", 1e-13), ("f32", 3e-6)):
        k = 0
        for n in SIZES:
            for sign in (-1, 1):
                x = lines[k]
                k += 1
                ref = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * n
                got = out[pos:pos + n]
                pos += n
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= tol, (prec, n, sign, err)
