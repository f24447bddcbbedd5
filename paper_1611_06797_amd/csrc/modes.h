// Arithmetic modes of the matrix-core contractions.
#pragma once

namespace ltmp2 {
enum { kF64 = 0, kF32 = 1, kBF16x3 = 2 };
}
