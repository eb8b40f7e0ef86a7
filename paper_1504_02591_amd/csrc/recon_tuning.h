// Tuning knobs of the transform kernels, written by paper_1504_02591_amd/autotune.py (a -D on the
// compiler command line overrides them).  Tiles: packed z column pairs, y-pass columns, x-pass
// rows per block; middle radix split of the 512- and 1024-point transforms.
// Chosen on a 512^3 correction pass (fastest per knob); ms per pass of each variant:
//   base                   3.1303
//   RECON_TILE_X=8         3.1340
//   RECON_TILE_Z=8         3.1527
//   RECON_TILE_X=2         3.1891
//   RECON_MID_512=2        3.2430
//   RECON_MID_512=1        3.2689
//   RECON_TILE_Y=8         3.5862
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
