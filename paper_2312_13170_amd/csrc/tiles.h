// Compiled tile shapes of each kernel family.  The host tuning table
// (tune.cpp) indexes these lists; the kernel files instantiate exactly these
// shapes.  The grouped kernels (grouped.hip) check at plan time that the
// candidates they share with the single-problem kernels have the same shape.

// {index, bm, bn, bk, waves_m, waves_n, split_k, prefetch depth}
// split_k: 1 none, > 1 split reduction into that many chunks, 0 stream-K
// (symmetric contractions only).  prefetch: main-loop mode 1-4; in the FP32
// GEMM list 5-7 are modes 1-3 with B transposed into LDS and 8 is the
// direct-to-LDS loop with a two-stage ring (K a multiple of the K-tile).
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
    X(26, 128, 64, 32, 4, 2, 1, 4)           \
    X(27, 128, 128, 32, 2, 2, 1, 3)          \
    X(28, 128, 128, 32, 2, 2, 1, 4)          \
    X(29, 128, 128, 64, 2, 2, 1, 2)          \
    X(30, 128, 128, 32, 4, 4, 1, 6)          \
    X(31, 128, 128, 32, 2, 4, 1, 6)          \
    X(32, 128, 128, 32, 2, 4, 1, 7)          \
    X(33, 128, 128, 32, 2, 2, 1, 7)          \
    X(34, 128, 128, 64, 2, 2, 1, 6)          \
    X(35, 128, 128, 64, 2, 4, 1, 5)          \
    X(36, 64, 128, 32, 2, 4, 1, 6)           \
    X(37, 64, 64, 32, 2, 2, 1, 6)            \
    X(38, 128, 128, 64, 2, 4, 1, 6)          \
    X(39, 128, 128, 64, 2, 2, 1, 7)          \
    X(40, 128, 128, 64, 4, 4, 1, 8)          \
    X(41, 128, 128, 64, 2, 4, 1, 8)          \
    X(42, 128, 128, 64, 2, 2, 1, 8)          \
    X(43, 64, 128, 64, 2, 4, 1, 8)           \
    X(44, 128, 128, 32, 4, 4, 1, 8)          \
    X(45, 128, 128, 32, 2, 4, 1, 8)          \
    X(46, 128, 128, 32, 2, 2, 1, 8)          \
    X(47, 256, 128, 32, 4, 2, 1, 4)          \
    X(48, 256, 128, 32, 4, 2, 1, 8)          \
    X(49, 128, 256, 32, 2, 4, 1, 8)          \
    X(50, 32, 32, 32, 1, 1, 1, 3)

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
    X(21, 64, 64, 32, 2, 2, 0, 2)            \
    X(22, 128, 128, 32, 2, 4, 1, 3)          \
    X(23, 64, 64, 32, 2, 2, 1, 3)            \
    X(24, 128, 128, 32, 4, 4, 0, 3)          \
    X(25, 128, 128, 32, 2, 4, 0, 4)          \
    X(26, 32, 32, 32, 1, 1, 1, 3)

// bf16 / fp16 matrix-core GEMM on pre-rounded operands; the last column is
// the LDS layout here (1: XOR-swizzled rows, 2: rows padded by 16 bytes,
// 3: layout 1 filled by direct HBM-to-LDS loads, 4: layout 3 with the next
// k step's operands read from LDS while the current step's matrix
// instructions run, 5: layout 4 with the direct loads issued between the
// matrix instructions, 6 / 7: layout 5 on a four / five stage ring).
// The split variant caps the layout at 4 (the interleaved loads spill its
// registers, and its stage holds both parts, so two stages fill the LDS).
// The split-bf16 variant caps the K-tile at 32.  Candidates 13 and 14 give
// each of four waves a 128 x 128 block (256 accumulator registers, one wave
// per SIMD): half the LDS fragment reads per matrix-core step of the
// eight-wave 128 x 64 blocks.
#define LI_GEMM_LP_CANDIDATES(X)             \
    X(0, 256, 256, 32, 2, 4, 1, 1)           \
    X(1, 128, 128, 64, 2, 2, 1, 1)           \
    X(2, 256, 128, 32, 2, 2, 1, 1)           \
    X(3, 128, 256, 32, 2, 2, 1, 1)           \
    X(4, 64, 64, 64, 2, 2, 1, 1)             \
    X(5, 256, 256, 32, 2, 4, 1, 2)           \
    X(6, 128, 128, 64, 2, 2, 1, 2)           \
    X(7, 256, 128, 32, 2, 2, 1, 2)           \
    X(8, 256, 256, 32, 2, 4, 1, 3)           \
    X(9, 128, 128, 32, 2, 2, 1, 3)           \
    X(10, 256, 128, 32, 2, 2, 1, 3)          \
    X(11, 128, 256, 32, 2, 2, 1, 3)          \
    X(12, 256, 256, 64, 2, 4, 1, 3)          \
    X(13, 256, 256, 64, 2, 2, 1, 3)          \
    X(14, 256, 256, 32, 2, 2, 1, 3)          \
    X(15, 256, 256, 32, 2, 4, 1, 4)          \
    X(16, 256, 256, 64, 2, 4, 1, 4)          \
    X(17, 256, 256, 64, 2, 2, 1, 4)          \
    X(18, 256, 256, 32, 2, 2, 1, 4)          \
    X(19, 256, 256, 32, 2, 4, 1, 5)          \
    X(20, 256, 256, 64, 2, 4, 1, 5)          \
    X(21, 256, 256, 64, 2, 2, 1, 5)          \
    X(22, 256, 256, 32, 2, 2, 1, 5)          \
    X(23, 256, 256, 32, 2, 4, 1, 6)          \
    X(24, 256, 256, 32, 2, 4, 1, 7)          \
    X(25, 256, 256, 32, 2, 2, 1, 6)          \
    X(26, 256, 256, 32, 2, 2, 1, 7)

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

// Shape classes of the grouped execution (grouped.hip), also the candidates
// of the tuning families LI_KERNEL_GROUPED_GEMM / LI_KERNEL_GROUPED_COV.
// Each class is one contraction kernel per problem kind whose tiles share
// the block tile; the main loop keeps two K-tiles in flight with the LDS
// operand reads pipelined across the barrier (mode 3) and loads rows of any
// alignment with 16-byte loads.  The GEMM and covariance candidates named
// are the single-problem candidates of the same shape, which the
// per-instance launch loop of a plan uses.
// {class, GEMM candidate, covariance candidate, block tile, BK, waves_m,
//  waves_n, main-loop mode}.  The 32 tile (one wave) wastes less of small
// problems on padding.
#define LI_GROUPED_CLASSES(X)      \
    X(0, 13, 22, 128, 32, 2, 4, 3) \
    X(1, 16, 23, 64, 32, 2, 2, 3)  \
    X(2, 50, 26, 32, 32, 1, 1, 3)
