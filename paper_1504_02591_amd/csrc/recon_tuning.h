// Tuning knobs of the transform kernels, written by paper_1504_02591_amd/autotune.py (a -D on the
// compiler command line overrides them).  Tiles: packed z column pairs, y-pass columns, x-pass
// rows per block; middle radix split of the 512- and 1024-point transforms; z tiles per block of
// the z iteration.
// Chosen on a 512^3 correction pass (fastest per knob); ms per pass of each variant:
//   base                   2.6144
//   RECON_TILE_Z=8         2.6168
//   RECON_TILE_X=2         2.6414
//   RECON_TILE_X=8         2.6496
//   RECON_MID_512=2        2.7548
//   RECON_MID_512=1        2.7652
//   RECON_TILE_Y=8         2.9666
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
#define RECON_Z_TPB 4
#endif
