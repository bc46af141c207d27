// Compiled tile shapes of each kernel family.  The host tuning table
// (tune.cpp) indexes these lists; the kernel files instantiate exactly these
// shapes.  The grouped kernels (grouped.hip) check at plan time that the
// candidates they share with the single-problem kernels have the same shape.

// {index, bm, bn, bk, waves_m, waves_n, split_k, prefetch depth}
// split_k: 1 none, > 1 split reduction into that many chunks, 0 stream-K
// (symmetric contractions only)
#define LI_GEMM_F32_CANDIDATES(X)            \
    X(0, 128, 128, 32, 2, 2, 1, 1)           \
    X(1, 128, 128, 16, 2, 2, 1, 1)           \
    X(2, 64, 64, 32, 2, 2, 1, 1)             \
    X(3, 128, 64, 32, 2, 2, 1, 1)            \
    X(4, 64, 128, 32, 2, 2, 1, 1)            \
    X(5, 128, 128, 32, 2, 4, 1, 1)           \
    X(6, 128, 128, 32, 2, 4, 1, 2)           \
    X(7, 128, 128, 32, 4, 4, 1, 1)           \
    X(8, 128, 128, 64, 2, 4, 1, 1)           \
    X(9, 128, 128, 32, 4, 4, 1, 2)           \
    X(10, 64, 64, 32, 2, 2, 1, 2)            \
    X(11, 128, 128, 64, 4, 4, 1, 1)          \
    X(12, 128, 128, 64, 2, 4, 1, 2)          \
    X(13, 128, 128, 32, 2, 4, 1, 3)          \
    X(14, 128, 128, 64, 2, 4, 1, 3)          \
    X(15, 128, 128, 32, 4, 4, 1, 3)          \
    X(16, 64, 64, 32, 2, 2, 1, 3)            \
    X(17, 128, 128, 32, 2, 4, 1, 4)          \
    X(18, 128, 128, 32, 4, 4, 1, 4)          \
    X(19, 64, 64, 32, 2, 2, 1, 4)            \
    X(20, 64, 64, 64, 2, 2, 1, 4)            \
    X(21, 64, 128, 32, 2, 4, 1, 2)           \
    X(22, 128, 64, 32, 4, 2, 1, 2)           \
    X(23, 64, 128, 32, 2, 4, 1, 3)           \
    X(24, 128, 64, 32, 4, 2, 1, 3)           \
    X(25, 64, 128, 32, 2, 4, 1, 4)           \
    X(26, 128, 64, 32, 4, 2, 1, 4)

// square block tiles only (upper-triangle enumeration)
#define LI_SYRK_F32_CANDIDATES(X)            \
    X(0, 128, 128, 32, 2, 2, 1, 1)           \
    X(1, 128, 128, 16, 2, 2, 1, 1)           \
    X(2, 64, 64, 32, 2, 2, 1, 1)             \
    X(3, 128, 128, 32, 2, 4, 1, 1)           \
    X(4, 64, 64, 32, 2, 2, 1, 2)             \
    X(5, 128, 128, 32, 2, 4, 1, 2)           \
    X(6, 128, 128, 32, 2, 4, 2, 1)           \
    X(7, 128, 128, 32, 2, 4, 4, 1)           \
    X(8, 128, 128, 32, 2, 2, 4, 1)           \
    X(9, 128, 128, 32, 2, 4, 7, 1)           \
    X(10, 128, 128, 32, 4, 4, 7, 2)          \
    X(11, 128, 128, 64, 4, 4, 7, 1)          \
    X(12, 128, 128, 64, 2, 4, 4, 1)          \
    X(13, 128, 128, 32, 4, 4, 7, 3)          \
    X(14, 128, 128, 32, 2, 4, 7, 3)          \
    X(15, 128, 128, 32, 4, 4, 7, 4)          \
    X(16, 128, 128, 32, 2, 4, 7, 4)          \
    X(17, 64, 64, 32, 2, 2, 1, 4)            \
    X(18, 128, 128, 32, 4, 4, 0, 2)          \
    X(19, 128, 128, 32, 2, 4, 0, 3)          \
    X(20, 128, 128, 32, 4, 4, 0, 4)          \
    X(21, 64, 64, 32, 2, 2, 0, 2)

// bf16 / fp16 matrix-core GEMM on pre-rounded operands; the last column is
// the LDS layout here (1: XOR-swizzled rows, 2: rows padded by 16 bytes).
// The split-bf16 variant caps the K-tile at 32.
#define LI_GEMM_LP_CANDIDATES(X)             \
    X(0, 256, 256, 32, 2, 4, 1, 1)           \
    X(1, 128, 128, 64, 2, 2, 1, 1)           \
    X(2, 256, 128, 32, 2, 2, 1, 1)           \
    X(3, 128, 256, 32, 2, 2, 1, 1)           \
    X(4, 64, 64, 64, 2, 2, 1, 1)             \
    X(5, 256, 256, 32, 2, 4, 1, 2)           \
    X(6, 128, 128, 64, 2, 2, 1, 2)           \
    X(7, 256, 128, 32, 2, 2, 1, 2)

// Row-form symmetric updates (syrk A A^T, syr2k A B^T + B A^T): square block
// tiles, operands with k contiguous.
#define LI_SYRK_ROWS_CANDIDATES(X)           \
    X(0, 128, 128, 32, 2, 2, 1, 1)           \
    X(1, 64, 64, 32, 2, 2, 1, 1)             \
    X(2, 128, 128, 32, 2, 4, 1, 3)           \
    X(3, 128, 128, 32, 2, 4, 2, 3)           \
    X(4, 128, 128, 32, 2, 4, 4, 3)           \
    X(5, 128, 128, 32, 4, 4, 4, 2)           \
    X(6, 128, 128, 32, 4, 4, 7, 2)           \
    X(7, 128, 128, 32, 2, 4, 7, 3)           \
    X(8, 128, 128, 32, 4, 4, 4, 4)           \
    X(9, 64, 64, 32, 2, 2, 4, 2)             \
    X(10, 64, 64, 32, 2, 2, 1, 3)            \
    X(11, 128, 128, 32, 4, 4, 2, 4)          \
    X(12, 128, 128, 32, 4, 4, 0, 2)          \
    X(13, 128, 128, 32, 2, 4, 0, 3)          \
    X(14, 64, 64, 32, 2, 2, 0, 2)            \
    X(15, 128, 128, 32, 4, 4, 0, 4)
