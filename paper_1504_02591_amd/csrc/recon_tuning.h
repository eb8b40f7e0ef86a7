// Tuning knobs of the transform kernels, written by paper_1504_02591_amd/autotune.py (a -D on the
// compiler command line overrides them).  Tiles: packed z column pairs, y-pass columns, x-pass
// rows per block; middle radix split of the 512- and 1024-point transforms; z tiles per block of
// the z iteration.
// Chosen on a 512^3 correction pass (fastest per knob); ms per pass of each variant:
//   RECON_Z_TPB=8          2.5736
//   base                   2.5814
//   RECON_TILE_X=2         2.5904
//   RECON_Z_TPB=2          2.5949
//   RECON_TILE_X=8         2.5954
//   RECON_Z_TPB=1          2.6240
//   RECON_TILE_Z=8         2.6522
//   RECON_MID_512=2        2.7369
//   RECON_MID_512=1        2.7386
//   RECON_TILE_Y=8         2.8554
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
#ifndef RECON_MID_1024
#define RECON_MID_1024 0
#endif
#ifndef RECON_Z_TPB
#define RECON_Z_TPB 8
#endif
#ifndef RECON_Z_DEFER
#define RECON_Z_DEFER 1
#endif
#ifndef RECON_Z_WAVE
#define RECON_Z_WAVE 0
#endif
// Per-size knobs (the 256^3 and 1024^3 grids; the general value until tuned at that size)
#ifndef RECON_TILE_Z_256
#define RECON_TILE_Z_256 RECON_TILE_Z
#endif
#ifndef RECON_TILE_Y_256
#define RECON_TILE_Y_256 RECON_TILE_Y
#endif
#ifndef RECON_TILE_X_256
#define RECON_TILE_X_256 RECON_TILE_X
#endif
#ifndef RECON_Z_TPB_256
#define RECON_Z_TPB_256 RECON_Z_TPB
#endif
#ifndef RECON_TILE_X_1024
#define RECON_TILE_X_1024 RECON_TILE_X
#endif
#ifndef RECON_Z_TPB_1024
#define RECON_Z_TPB_1024 RECON_Z_TPB
#endif
// Deposit launch shapes, timed on the 512^3 survey catalogues (ms per reconstruction, both catalogues):
//   brick accumulation threads per brick  256: 0.640   512: 0.522   1024: 0.585
//   binning blocks (one 128 KB LDS histogram each)  1024: 1.018   512: 0.951   256: 0.915
//   objects per loop trip (deposit + randoms' shift)  2: 0.512 + 1.025   4: 0.497 + 1.025   8: 0.510 + 1.062
//   reorder after the brick-order shift, chunks of one block (shift stage, both catalogues)
//     per_x apart: 1.096   adjacent (one trip per block), 2 / 4 / 8 chunks: 0.980 / 0.983 / 0.980
#ifndef RECON_BRICK_NT
#define RECON_BRICK_NT 512
#endif
#ifndef RECON_BIN_BLOCKS
#define RECON_BIN_BLOCKS 256
#endif
#ifndef RECON_OBJ_BATCH
#define RECON_OBJ_BATCH 4
#endif
