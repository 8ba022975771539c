// fused.h - LDS-staged fusion of consecutive gates: the data a fused pass hands
// to its kernel.
//
// A fused pass picks a set S of qudits: the lowest qudits (so that the tile is
// made of contiguous runs of L amplitudes) plus every target of the gates in the
// pass. A tile is the M_S = prod_{q in S} d_q amplitudes that share one value of
// every digit outside S; tiles are disjoint and every gate of the pass maps each
// tile to itself, because each gate's classes (Sec. 2.3) only vary target digits.
// A workgroup loads one tile into LDS, applies the gates of the pass in order to
// the tile, and writes the tile back once, so the pass costs one HBM read and
// one HBM write of the state instead of one per gate.
//
// Inside the tile, amplitudes are ordered by the S digits in increasing qudit
// order, so the tile is itself a small mixed-radix register and each gate gets
// an ordinary class plan over it. A control on a qudit inside S is a control of
// that tile-local plan; a control on a qudit outside S is constant over a tile
// and becomes a per-tile predicate on the tile's base address.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "plan.h"

namespace qd {

constexpr int kTileMaxSeg = 8;      // free segments of a batched item's tile-index decoder
constexpr int kFuseMaxM = 16;       // class size (dense) / active count (monomial) inside a tile
constexpr size_t kPassBlobMax = 1536u << 10;  // device data of one fused pass (fits a 2 MB staging slot)
constexpr int kMaxOuterCtl = 8;     // controls outside S per gate

// A gate's classes inside a tile are the same for every tile, so every pass
// ships their tile-local bases as a uint16 table (a tile has at most 32768
// amplitudes) instead of decoding them on the device.

// Two consecutive dense gates on disjoint targets, both with classes of at most
// kPairMaxM amplitudes and no controls, share one descriptor: a thread reads the
// joint class (the M1 x M2 amplitudes over both gates' targets, local index
// a1 + M1 a2) from LDS once, applies the first gate to each of its M2 sub-classes
// and the second to each of its M1 sub-classes in registers, and writes it back
// once. Every amplitude sees the same operations as with the two gates applied
// one after the other, so the result is bitwise the same, with half the LDS
// traffic.
constexpr int32_t kDensePair = 8;   // TileGate::kind of a pair (distinct from the Category values)
constexpr int kPairMaxM = 4;

// Consecutive dense gates with the same targets (in the same order) and the
// same controls act on the same classes: a chain of them shares one
// descriptor. A thread reads a class from LDS once, applies the gates one after
// the other in registers (each row with the single-gate arithmetic) and writes
// it back once: bitwise the gate-by-gate result, with one LDS round trip and
// one barrier for the whole chain.
constexpr int32_t kDenseChain = 9;  // TileGate::kind of a chain; M2 = its length, the matrices follow each other
constexpr int kChainMaxM = 3;  // at 4, one gate's matrix (64 scalar registers in complex128) spills
constexpr int kChainMaxLen = 16;

// A register block: a run of gates with no controls inside the tile (controls
// outside it are constant per tile: see BlockGate) whose targets all lie in a set T
// of at most 3 tile qudits with at most kBlockMaxJ (complex64) or
// kBlockMaxJ128 (complex128) amplitudes in the joint class over T. A thread reads
// a joint class (the amplitudes that differ only in the T digits) from LDS
// once, applies every gate of the block to its sub-classes in registers with
// the single-gate arithmetic (dense rows as dense_row, phases and shifts as the
// monomial update), and writes it back once: bitwise the gate-by-gate result,
// with one LDS round trip and one barrier for the whole block. The joint index
// runs over T in the block's shape order (dims ascending; ties by tile
// position), first position least significant; TileGate::off holds the tile
// offsets of the J joint members, one_mask the shape id (kBlockShapes), M2 the
// number of gates, u_off their BlockGate records (then their BlockOuter records)
// and dst[0] how many of them have controls outside the tile.
constexpr int32_t kBlock = 10;      // TileGate::kind of a register block
constexpr int kBlockMaxJ = 16;
constexpr int kBlockMaxJ128 = 12;  // 128 VGPRs in the tile kernels (16 needs 166: fewer waves per SIMD)
constexpr int kBlockMaxGates = 32;

// Block shapes: the dims of T in joint order (1 pads), joint size at most 16.
constexpr int kBlockShapeCount = 19;
constexpr int kBlockShapes[kBlockShapeCount][3] = {
    {2, 1, 1}, {3, 1, 1}, {4, 1, 1}, {5, 1, 1}, {6, 1, 1}, {7, 1, 1},
    {2, 2, 1}, {2, 3, 1}, {2, 4, 1}, {2, 5, 1}, {2, 6, 1}, {2, 7, 1}, {3, 3, 1}, {3, 4, 1}, {3, 5, 1}, {4, 4, 1},
    {2, 2, 2}, {2, 2, 3}, {2, 2, 4}};

// One gate of a block: code = kind * 16 + p * 4 + q, p (and q) the joint
// positions of its first (and second) target.
enum BlockKind { kBlkDense1 = 0, kBlkDiag1 = 1, kBlkShift1 = 2, kBlkDense2 = 3 };
struct BlockGate {
    int32_t code;
    uint32_t u_off;     // blob offset: dense: the M x M matrix; phase: one factor per local index
    uint32_t one_mask;  // phase: bit a set if local index a keeps its amplitude (factor exactly 1)
    int32_t shift;      // shift: |a> -> |a + shift mod d>
};

// A block gate may have up to kBlockMaxOuter controls on qudits outside the tile:
// constant over a tile, they decide once per tile whether the gate acts on it
// (Sec. 2.4), as for a descriptor's outer controls. Such a gate has a BlockOuter
// record; a block's records follow its BlockGate array (TileGate::dst[0] of
// them, at most kBlockMaxOuterGates).
constexpr int kBlockMaxOuter = 2;
constexpr int kBlockMaxOuterGates = kBlockMaxGates;
struct BlockOuter {
    uint32_t gate;      // index of the gate in the block
    int32_t n_outer;    // the gate acts on a tile iff for every l < n_outer:
    uint32_t oc_dim[kBlockMaxOuter];   //   (tile base / oc_stride[l]) mod oc_dim[l] == oc_val[l]
    uint32_t oc_val[kBlockMaxOuter];
    FastDiv<uint32_t> oc_sdiv[kBlockMaxOuter];  // the same divisions for 32-bit tile bases
    FastDiv<uint32_t> oc_ddiv[kBlockMaxOuter];
    uint64_t oc_stride[kBlockMaxOuter];
};

struct TileGate {
    // Fields every gate reads come first (the kernel reads them through the
    // scalar cache: fewer cache lines per descriptor).
    int32_t kind;        // kDense, kDensePair, kDenseChain, kBlock, or kMonomial for monomial and diagonal gates
    int32_t M;           // dense, chain: class size; pair: class size of the first gate; monomial: active entries
    int32_t M2;          // pair: class size of the second gate (its U follows the first's in the blob);
                         // chain: number of gates
    uint32_t n_classes;                 // classes of the gate inside one tile
    uint32_t bases_off;                 // byte offset of the uint16 class bases in the blob
    uint32_t u_off;                     // byte offset of U (dense) or the factors (monomial) in the blob
    uint32_t one_mask;                  // monomial: bit i set if factor i is exactly 1
    int32_t n_outer;                    // controls outside S
    uint32_t off[kFuseMaxM];            // dense, pair, chain: member offsets; monomial: source offsets
    uint32_t dst[kFuseMaxM];            // monomial: destination offsets
    uint64_t oc_stride[kMaxOuterCtl];   // the gate runs on a tile iff for every l:
    uint32_t oc_dim[kMaxOuterCtl];      //   (tile base / oc_stride[l]) mod oc_dim[l] == oc_val[l]
    uint32_t oc_val[kMaxOuterCtl];
};

// Scalar kernel arguments of a fused pass. The device arrays (gate descriptors,
// gate data, run offsets) are separate `const __restrict__` kernel parameters so
// that the compiler may read them through the scalar cache.
template <typename I>
struct FusedArgs {
    Decode<I> outer;                    // tile id -> base address of the tile
    uint32_t tile;                      // amplitudes per tile (M_S)
    uint32_t L;                         // contiguous run length
    uint32_t chunks_per_run;            // ceil(L / 64): wavefront-sized pieces of a run
    uint32_t nchunks;                   // runs * chunks_per_run
    FastDiv<uint32_t> cdiv;             // division by chunks_per_run
    int32_t ngates;
};

// One (state, fused pass) of a batched round. Workgroups [first_block,
// first_block + n_tiles) of the launch process this item's tiles.
struct BatchItem {
    uint64_t psi;                        // device address of the state's amplitudes
    Decode<uint32_t, kTileMaxSeg> outer; // tile id -> tile base
    uint32_t tile, L, chunks_per_run, nchunks;
    FastDiv<uint32_t> cdiv;
    int32_t ngates;
    uint32_t gates_off;                  // byte offsets into the round's blob
    uint32_t run_off_off;
    uint32_t first_block;
};

}  // namespace qd
