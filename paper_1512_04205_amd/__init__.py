"""MI355X-native compressed dynamic mode decomposition (cDMD) for video background
modeling: a HIP library for gfx950 behind a C ABI (include/cdmd.h), and this thin
Python binding.  Importing the package loads libcdmd.so and fails if it is not built.
"""
from ._binding import (  # noqa: F401
    CdmdError, Model, Batch, optimal_rank, process_video, VideoExecutor, load_library, unpack_mask,
    mask_words, mask_median3, LIB_PATH, EXPORTED,
    MLP_NPARAM, MLP_NOALLOC_MAX_BATCH, mlp_grad, mlp_train, mlp_train_noalloc, mlp_forward,
    U8, F32, SKETCH_GAUSSIAN, SKETCH_SPARSE, SKETCH_SPIXEL, SKETCH_SRFT, PREC_FP32, PREC_BF16, PREC_FP8,
    SEL_OMP, SEL_ZERO_MODE, SEL_OMEGA, SEL_EXPLICIT, SEL_ALL, AMP_FULL, AMP_COMPRESSED,
    OK, E_INVALID_ARG, E_UNSUPPORTED, E_OUT_OF_MEMORY, E_DEVICE, E_RANK_DEFICIENT, E_NUMERIC,
    E_STATE,
)

load_library()
