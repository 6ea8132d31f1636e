// Arithmetic of the persistent launch's grid-barrier tree: the blocks found
// on one XCD (by the census at the start of the launch) form groups of G in
// the order of their census rank; the last block of a group to arrive
// arrives at its XCD, the last group of an XCD arrives at the global
// counter, whose target is the number of XCDs in use.  Plain constexpr C++:
// the device code and a CPU check program include it alike.
#pragma once

namespace msb {
namespace tree {

struct Group {
    int g;       // the block's group on its XCD
    int ng;      // groups on that XCD
    int gsize;   // blocks in the block's group
};

// block of census rank k among the nx blocks of its XCD, groups of G
constexpr Group group_of(int k, int nx, int G) {
    const int g = k / G;
    const int ng = (nx + G - 1) / G;
    return Group{g, ng, g == ng - 1 ? nx - g * G : G};
}

}  // namespace tree
}  // namespace msb
