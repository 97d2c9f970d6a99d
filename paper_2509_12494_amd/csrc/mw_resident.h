// Device-resident request loop of the serving runtime: one persistent kernel
// takes transform, product and BLAS requests of one- and two-word moduli from
// a ring in mapped host memory and runs their tiles, so a request costs no
// kernel launch.
//
// Protocol (host = the server's scheduler, device = the kernel):
//  * The host writes entry e (global number) into ring slot e mod kResRing of
//    the mapped host block, then publishes it by storing tail = e + 1.
//  * Workgroup 0 of the kernel (the dispatcher) polls tail.  For each new
//    entry it copies the descriptor into device memory and writes one word
//    per tile into the tile ring: word g (global tile number) is
//    g << 24 | slot << 12 | tile, stored at g mod kResTileRing.
//  * Every other workgroup (a worker, one per compute unit) claims the next
//    global tile number g with an atomic add, waits until word g carries tag
//    g, then runs that tile and adds one to the entry's completed-tile count.
//    A tile of phase k > 0 first waits until the slot's phase word reaches k;
//    the tile whose count completes phase k - 1 stores it.  Tiles are
//    numbered phase by phase, so the earliest unfinished tile never waits on
//    a later one and the loop cannot deadlock.  The workgroup that completes
//    the entry's last tile stores seq + 1 (bit 63: a dependency wait timed
//    out) into the slot's done word in host memory, which the host polls.
//  * Tiles of different workgroups meet through device memory on different
//    XCDs, whose L2 caches are not coherent with each other within a kernel.
//    A tile invalidates its compute unit's L1 and its XCD's L2 once (agent-
//    scope acquire, by one lane) before it reads the descriptor, the
//    request's inputs and its twiddle tables.  The residues tiles write (a
//    phase's outputs, read by the next phase, and the request's results)
//    move by device-scope loads and stores, so no L2 write-back is needed:
//    every wave waits for its own stores before the count is raised.
//  * Device-scope accesses to one 128-byte line are served one after
//    another, so the words that many workgroups touch at once -- the claim
//    cursor, the stop and heartbeat words, the completion count, each slot's
//    phase word -- sit on lines of their own, and idle workers read the stop
//    and heartbeat words on every 8th poll only.
//  * Every wait is bounded: workers leave when the dispatcher sets the stop
//    word, or when its heartbeat has not moved for the stall bound (a
//    dispatcher that is not running); the dispatcher leaves when the host
//    asks it to (after draining) or when every entry it took is complete and
//    no new one arrived for the idle time, and also when entries are pending
//    but none has completed for the stall bound; a dependency wait gives up
//    (marking the entry failed) after the wait bound.  The host relaunches
//    the kernel when it publishes an entry and finds the kernel gone, and
//    fails the entries an ended kernel took but did not complete.
//  * Yielding: streams share the device's few hardware queues, and a kernel
//    queued behind the loop on its queue cannot start before the loop ends.
//    When work the host launched elsewhere stays unfinished too long, the
//    host sets the yield word: the dispatcher takes no new entry, the loop
//    ends once the entries it took are complete, whatever waited behind it
//    runs, and the host launches the loop again after it.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "mw_blas_elem.h"
#include "mw_exec.h"

namespace mw {

constexpr u32 kResRing = 1024;              // entries in the ring (power of two, <= 4096)
constexpr u32 kResTileRing = 1u << 20;      // tile words (power of two)
constexpr u32 kResMaxTiles = 4096;          // tiles per entry (12 bits of a tile word)
constexpr u32 kResLds = 48 * 1024;          // dynamic LDS of a worker: the largest tile it takes
constexpr u32 kResBlasChunk = 4 * 256;      // residues per BLAS tile
constexpr u32 kResMaxLog2N = 17;            // largest transform the loop takes (a plan's largest)
// By default every request the loop can take goes to it; a smaller bound
// (mw_server_config.resident_max_tiles) sends larger requests to the slot
// path.  A slot-path launch can land on the loop's hardware queue and then
// waits for the loop to yield, and the loop is faster than the slot path for
// requests of every size it takes (measured on MI355X, 20 K requests/s
// Poisson stream).
constexpr u32 kResRouteTiles = kResMaxTiles;
constexpr u64 kResTagMask = (u64(1) << 40) - 1;

enum { RES_NTT = 0, RES_BLAS = 1 };

// One request.  Transforms and products: `job` (as the batched executor's)
// and the constants of its width; BLAS: op, length, operands and the modulus
// (m4.M / m2.M) with the axpy scalar.
struct alignas(16) ResEntry {
  u64 seq;              // global entry number
  u32 kind;             // RES_NTT / RES_BLAS
  u32 limbs;            // 1 or 2
  u32 total;            // tiles
  u32 nphases;
  u32 prefix[4];        // tiles before phase k; prefix[nphases] = total
  u32 blas_op;          // OP_ADD .. OP_AXPY (c = alpha*a + b for axpy)
  u32 pad0;
  u64 n;                // BLAS length
  u64 a, b, c;          // BLAS operands and output
  JobDesc job;
  ModConst<4> m4;       // constants of a two-word modulus
  ModConst<2> m2;       // one-word
  Scalar<4> s4;
  Scalar<2> s2;
};
static_assert(sizeof(ResEntry) % 16 == 0, "entries are copied in 16-byte units");

// Device control words, reset by the host before each launch.  The words
// that idle workers poll (stop, beat), the claim cursor and the completion
// count sit on 128-byte lines of their own: device-scope accesses to one line
// queue behind each other in memory.
struct ResCtl {
  alignas(128) u64 gcursor;   // next global tile number to claim
  alignas(128) u32 stop;      // dispatcher -> workers: leave
  u32 beat;                   // dispatcher's heartbeat, raised on every poll
  alignas(128) u64 completed; // entries completed (cumulative over launches)
  alignas(128) u32 exited;    // workers that have left
  u32 error;                  // a dependency wait timed out
};

// Device memory of the loop (one allocation).
constexpr u32 kResLineWords = 128 / sizeof(u32);
struct ResDevBlock {
  ResCtl ctl;
  u32 dcount[kResRing];           // tiles completed of the slot's entry
  u32 dfail[kResRing];            // the slot's entry had a failed wait
  // phases of the slot's entry complete, one 128-byte line per slot: the
  // waiting tiles of the next phase poll this word, not the count that the
  // running tiles raise
  u32 dphase[kResRing * kResLineWords];
  ResEntry dent[kResRing];        // descriptors, copied by the dispatcher
  u64 tiles[kResTileRing];        // tile words
};
static_assert(offsetof(ResDevBlock, dfail) == offsetof(ResDevBlock, dcount) + sizeof(u32) * kResRing &&
                  offsetof(ResDevBlock, dphase) == offsetof(ResDevBlock, dfail) + sizeof(u32) * kResRing,
              "the per-slot words are cleared as one range");
static_assert(offsetof(ResDevBlock, dphase) % 128 == 0, "one line per slot");

// Mapped pinned host memory of the loop.
struct ResHost {
  u64 tail;                       // host: entries published
  u64 consumed;                   // device: entries the dispatcher has taken
  u32 stop;                       // host: leave once every entry is complete
  u32 yield;                      // host: take no new entry; leave once every one taken is complete
  u32 pad[2];
  ResCtl ctl_init;                // staging of the control reset before a launch
  u64 done[kResRing];             // device: seq + 1 of the slot's last completed entry
  ResEntry ring[kResRing];
};

struct ResParams {
  ResHost* host;                  // device address of the mapped block
  ResDevBlock* dev;
  u64 start_entry;                // first entry this launch takes
  u64 gstart;                     // global number of that entry's first tile
  u64 idle_ticks;                 // dispatcher's idle time before it leaves (wall-clock ticks)
  u64 wait_ticks;                 // bound of a dependency wait
  u64 stall_ticks;                // bound without progress (see the protocol)
};

// Launches the loop with `grid` workgroups (workgroup 0 dispatches) on s.
hipError_t resident_launch(const ResParams& p, u32 grid, hipStream_t s);

}  // namespace mw
