// Tuning knobs of the transform kernels, written by paper_1504_02591_amd/autotune.py (a -D on the
// compiler command line overrides them).  Tiles: packed z column pairs, y-pass columns, x-pass
// rows per block; middle radix split of the 512- and 1024-point transforms; z tiles per block of
// the z iteration; wave-local z iteration at 512^3.  The general knobs are timed at 512^3 and
// serve every size without its own; the _256 and _1024 knobs are timed at those sizes.
// Chosen on a 256^3 correction pass of a batch of 64 (fastest per knob); ms per pass of each variant:
//   RECON_Z_TPB_256=4      18.3334
//   RECON_Z_TPB_256=1      18.3340
//   RECON_TILE_X_256=8     18.3761
//   base                   18.4052
//   RECON_TILE_X_256=2     18.4290
//   RECON_Z_TPB_256=2      18.4743
//   RECON_TILE_Z_256=8     18.5960
//   RECON_TILE_Y_256=8     20.6149
// Chosen on a 512^3 correction pass (fastest per knob); ms per pass of each variant:
//   base                   2.4034
//   RECON_Z_TPB=4          2.4174
//   RECON_TILE_X=2         2.4249
//   RECON_TILE_X=8         2.4291
//   RECON_Z_TPB=2          2.4547
//   RECON_MID_512=2        2.4941
//   RECON_MID_512=1        2.4949
//   RECON_Z_TPB=1          2.4980
//   RECON_Z_WAVE=0         2.4997
//   RECON_TILE_Z=8         2.5664
//   RECON_TILE_Y=8         2.7006
// Chosen on a 1024^3 correction pass (fastest per knob); ms per pass of each variant:
//   RECON_TILE_X_1024=2    28.2326
//   base                   29.0081
//   RECON_Z_TPB_1024=4     29.1065
//   RECON_TILE_X_1024=8    29.3792
//   RECON_MID_1024=1       29.5875
//   RECON_Z_TPB_1024=2     29.6346
//   RECON_MID_1024=2       29.7253
//   RECON_Z_TPB_1024=1     30.3946
#pragma once
#ifndef RECON_TILE_Z
#define RECON_TILE_Z 16
#endif
#ifndef RECON_TILE_Y
#define RECON_TILE_Y 16
#endif
#ifndef RECON_TILE_X
#define RECON_TILE_X 4
#endif
#ifndef RECON_MID_512
#define RECON_MID_512 0
#endif
#ifndef RECON_Z_TPB
#define RECON_Z_TPB 8
#endif
#ifndef RECON_Z_WAVE
#define RECON_Z_WAVE 1
#endif
#ifndef RECON_TILE_Z_256
#define RECON_TILE_Z_256 16
#endif
#ifndef RECON_TILE_Y_256
#define RECON_TILE_Y_256 16
#endif
#ifndef RECON_TILE_X_256
#define RECON_TILE_X_256 8
#endif
#ifndef RECON_Z_TPB_256
#define RECON_Z_TPB_256 4
#endif
#ifndef RECON_TILE_X_1024
#define RECON_TILE_X_1024 2
#endif
#ifndef RECON_MID_1024
#define RECON_MID_1024 0
#endif
#ifndef RECON_Z_TPB_1024
#define RECON_Z_TPB_1024 8
#endif
// Deposit launch shapes, timed on the 512^3 survey catalogues (ms per reconstruction, both catalogues):
//   brick accumulation threads per brick  256: 0.640   512: 0.522   1024: 0.585
//   binning blocks (one 128 KB LDS histogram each)  1024: 1.018   512: 0.951   256: 0.915
//   objects per loop trip (deposit + randoms' shift)  2: 0.512 + 1.025   4: 0.497 + 1.025   8: 0.510 + 1.062
//   reorder after the brick-order shift, chunks of one block (shift stage, both catalogues)
//     per_x apart: 1.096   adjacent (one trip per block), 2 / 4 / 8 chunks: 0.980 / 0.983 / 0.980
// Non-temporal hint on the transform passes' spectrum accesses (bit 0 stores, bit 1 loads), timed on
// the 512^3 survey reconstruction (plain start, 6 passes, ms per reconstruction): 0: 20.30 / 20.46,
// 1: 19.71, 2: 19.96, 3: 19.41 / 19.45 (two runs; Psi bit-identical).  The same hint on the deposit's
// scattered brick-ordered copy made the binning 2.4x slower (0.79 -> 1.92 ms) and is not used.
// At 1024^3 (y tiles of 8 columns: half-line row segments) hinted loads made the y passes slower
// (fan-out 6.25 -> 7.05 ms, fan-in 5.88 -> 6.90 ms) while the z and x passes gained (8.80 -> 8.32,
// 6.09 -> 5.95 ms): the y passes hint their loads only at tiles of 16 columns or more.
// Binning above 512^3 (more bricks than one LDS histogram holds): per-block windows of the LDS
// histogram centred on the chunk's first object (RECON_BIN_WINDOW=1) instead of global atomics for
// every object: 1024^3 precision-study reconstruction (1.07e9 lattice particles) 773.7 -> 631.8 ms.
#ifndef RECON_X_WAVES
#define RECON_X_WAVES 0
#endif
#ifndef RECON_Z_DEFER
#define RECON_Z_DEFER 1
#endif
#ifndef RECON_BRICK_NT
#define RECON_BRICK_NT 512
#endif
#ifndef RECON_BIN_BLOCKS
#define RECON_BIN_BLOCKS 256
#endif
#ifndef RECON_OBJ_BATCH
#define RECON_OBJ_BATCH 4
#endif
#ifndef RECON_STREAM
#define RECON_STREAM 3
#endif
#ifndef RECON_BIN_WINDOW
#define RECON_BIN_WINDOW 1
#endif
