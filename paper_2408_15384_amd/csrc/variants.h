// Compiled tile variants of each method: X(id, BM, BN, BK, WM, WN), the
// workgroup tile BM x BN, its K step BK and the per-wave sub-tile WM x WN.
// The variant id is what the autotuner stores and mm_gemm_variant takes; the
// single-problem and grouped kernels instantiate the same lists, so a variant
// computes every tile the same way in both.
#pragma once

// Dense variants carry a seventh field, S: 0 for the register-staged tile, or
// 10 + b for the direct global-to-LDS tile with a ring of b buffers (which
// falls back to the register-staged tile for problems it cannot take).
#define MM_F64_VARIANTS(X)            \
    X(0, 128, 128, 16, 64, 64, 0)     \
    X(1, 64, 64, 16, 32, 32, 0)       \
    X(2, 256, 128, 16, 64, 64, 0)     \
    X(3, 128, 64, 16, 64, 32, 0)      \
    X(4, 256, 128, 16, 64, 64, 13)    \
    X(5, 128, 128, 16, 64, 64, 13)    \
    X(6, 64, 64, 16, 32, 32, 13)      \
    X(7, 64, 64, 16, 32, 32, 12)      \
    X(8, 128, 64, 16, 64, 32, 13)     \
    X(9, 32, 32, 16, 16, 16, 13)      \
    X(10, 32, 32, 16, 16, 16, 0)      \
    X(11, 128, 256, 16, 64, 64, 13)   \
    X(12, 256, 128, 16, 64, 64, 12)   \
    X(13, 64, 64, 16, 32, 32, 14)     \
    X(14, 32, 32, 16, 16, 16, 14)     \
    X(15, 256, 128, 16, 64, 32, 12)   \
    X(16, 64, 32, 16, 32, 16, 12)     \
    X(17, 64, 64, 32, 16, 16, 12)     \
    X(18, 128, 128, 32, 32, 32, 12)   \
    X(19, 32, 32, 32, 16, 16, 12)

#define MM_F32_VARIANTS(X)            \
    X(0, 128, 128, 16, 64, 64, 0)     \
    X(1, 64, 64, 16, 32, 32, 0)       \
    X(2, 256, 128, 16, 64, 64, 0)     \
    X(3, 128, 128, 32, 64, 64, 0)     \
    X(4, 256, 128, 32, 64, 64, 13)    \
    X(5, 256, 128, 16, 64, 64, 13)    \
    X(6, 64, 64, 32, 32, 32, 13)      \
    X(7, 64, 64, 16, 32, 32, 13)      \
    X(8, 64, 64, 32, 32, 32, 12)      \
    X(9, 128, 64, 32, 64, 32, 13)     \
    X(10, 32, 32, 32, 16, 16, 0)      \
    X(11, 256, 128, 16, 64, 64, 12)   \
    X(12, 256, 128, 32, 64, 64, 12)   \
    X(13, 256, 128, 32, 64, 32, 12)   \
    X(14, 256, 256, 32, 64, 64, 12)   \
    X(15, 32, 64, 32, 16, 32, 12)

// Split variants carry a seventh field, S: 1 or 2 register stages of global
// prefetch, or 10 + b: a ring of b LDS buffers fed by direct global-to-LDS
// loads (BK 32) -- all three read bfloat16 planes made by a split pass -- or
// 20: the fused tile, which reads the FP32 operands and splits them on the
// way into LDS (BK 32, no plane pass, no workspace); 20 + r: the fused tile
// with buffer loads and r K steps in flight in registers (64-byte LDS rows);
// 30 + r: the same with paired 128-byte LDS lines (one K step in flight:
// two measured no faster on grouped batches and at 1024, and cost
// occupancy where registers bound it).  A direct ring deeper
// than LDS holds for the method's planes is made shallower (variant 14 is a
// 3-buffer ring with 2 planes, a 2-buffer one with 3).
#define MM_SPLIT_VARIANTS(X)          \
    X(0, 128, 128, 32, 64, 64, 1)     \
    X(1, 64, 64, 32, 32, 32, 1)       \
    X(2, 128, 64, 32, 64, 32, 1)      \
    X(3, 128, 128, 32, 64, 32, 1)     \
    X(4, 128, 128, 32, 64, 32, 2)     \
    X(5, 64, 64, 32, 32, 32, 2)       \
    X(6, 128, 128, 32, 64, 32, 13)    \
    X(7, 128, 128, 32, 64, 64, 13)    \
    X(8, 64, 64, 32, 32, 32, 13)      \
    X(9, 256, 128, 32, 64, 64, 12)    \
    X(10, 64, 64, 32, 32, 32, 20)     \
    X(11, 128, 64, 32, 64, 32, 20)    \
    X(12, 128, 128, 32, 64, 32, 20)   \
    X(13, 128, 128, 32, 64, 64, 20)   \
    X(14, 256, 128, 32, 64, 64, 13)   \
    X(15, 64, 64, 32, 32, 32, 31)     \
    X(16, 128, 64, 32, 64, 32, 31)    \
    X(17, 64, 64, 32, 32, 32, 21)     \
    X(18, 128, 64, 32, 64, 32, 21)

// Size-class pairs of grouped launches: X(pair, small, large, pct).  Grouped
// variant id MM_PAIR_BASE + pair runs each problem of a batch on one of two
// variants of the same workgroup size: the small one when its tiles execute
// at most pct % of the large one's padded work (edge and K padding), else the
// large one.  Split pairs are ring-fused variants (no plane pass).
#define MM_F64_PAIRS(X)    \
    X(0, 16, 7, 90)        \
    X(1, 16, 6, 90)        \
    X(2, 14, 7, 80)
#define MM_F32_PAIRS(X)    \
    X(0, 15, 8, 90)        \
    X(1, 15, 8, 80)
#define MM_SPLIT_PAIRS(X)  \
    X(0, 15, 16, 90)       \
    X(1, 15, 16, 75)       \
    X(2, 17, 18, 90)       \
    X(3, 17, 18, 75)
