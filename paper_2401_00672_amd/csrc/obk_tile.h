// The sweep tile: the unit of work of the sweep kernels, shared by the host
// code that builds tiles and the device code that runs them.
#pragma once

#include <cstdint>

namespace obk {

// A tile is a contiguous range of "segments" (rows of a group in phase R,
// touched columns of a group in phase S) whose entries are reduced by one
// workgroup.  seg_begin/seg_end index segments, ent_begin/ent_end entries.
struct Tile {
    int32_t seg_begin, seg_end;
    int64_t ent_begin, ent_end;
};
constexpr int kTileThreads = 256;        // threads per tile (one sub-block)
constexpr int kTileSegs = 256;           // rows (columns) per tile, 1 per thread
constexpr int kTileEntries = 2048;       // entries staged per chunk (8 per thread)

}  // namespace obk
