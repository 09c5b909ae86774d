// Tile shapes chosen by paper_2107_03958_amd/autotune.py on MI355X (gfx950),
// timing the three apply passes at n = 2048; one parameter changed at a time
// from the previous shapes, kept when more than 1% faster.  WS_ERF64 (the
// forward real row pass's own elements per thread) was split from WS_ER64 after
// a sweep showed ER 16 faster for that pass alone (25.6 / 24.6 against
// 27.0 / 27.4 us per density at n = 2048, two runs each).  WS_ER64 went from
// 8 to 16 once the row passes issued all of a tile's loads before the first
// wait: FP64 inverse rows 24.7-24.8 -> 23.8-24.0 us per density at n = 2048
// (three runs), period-3 inverse rows at n = 1024 12.9 -> 10.0-10.1.
#pragma once
#ifndef WS_CB32
#define WS_CB32 2
#endif
#ifndef WS_CB64
#define WS_CB64 2
#endif
// WS_CHUNK_BYTES: 192 MiB (3 FP64 densities at n = 2048) measured 2-4% above
// 128 MiB (2) and 256 MiB (4) for the 32-density FP64 and FP32 steps at n = 2048.
#ifndef WS_CHUNK_BYTES
#define WS_CHUNK_BYTES (192u<<20)
#endif
#ifndef WS_CPB32
#define WS_CPB32 1
#endif
#ifndef WS_CPB64
#define WS_CPB64 1
#endif
#ifndef WS_EC32
#define WS_EC32 16
#endif
#ifndef WS_EC64
#define WS_EC64 16
#endif
#ifndef WS_ER32
#define WS_ER32 16
#endif
#ifndef WS_ER64
#define WS_ER64 16
#endif
#ifndef WS_ERF64
#define WS_ERF64 16
#endif
#ifndef WS_MIN_BLOCK
#define WS_MIN_BLOCK 64
#endif
#ifndef WS_RPB32
#define WS_RPB32 2
#endif
#ifndef WS_RPB64
#define WS_RPB64 2
#endif
