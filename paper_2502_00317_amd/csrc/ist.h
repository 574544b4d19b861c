// ist.h -- launch interface of the Induced Subgraph Trie listing kernel.
#pragma once

#include "internal.h"

// Parameters of one launch of k_list_ist: roots [root_begin, root_begin +
// nroots) of roots[], every root's records at out[rec_off[i] .. + rec_cnt[i]).
struct IstParams {
  const int32_t* dptr;
  const int32_t* dcol;
  const int32_t* orig;
  const int32_t* roots;
  const u64* gw;
  int k, prune, memo, fingerprint;
  int32_t root_begin, nroots;
  unsigned* cursor;
  const u64* rec_off;
  const u64* rec_cnt;
  int32_t* out;
  int32_t drows;
  char* trie;             // per-wave regions of trie_stride bytes
  u64 trie_stride;
  uint32_t node_cap;      // nodes per wave (< 2^24), node 0 the trie's root
  u64 hmask;              // hash slots per wave - 1 (a power of two minus one)
  u64 epoch_base;         // root i of the launch uses epoch epoch_base + i
  u64* wave_out;          // 16 words per wave
  int* err;               // set if a root's records disagree with its count
  // inspection (grid of one wave, one root): after the root, ListingIST of
  // the node whose set is ret_key, with l = ret_l and C = {root}, into
  // out[ret_off .. ret_off + ret_cap)
  int inspect;
  int ret_l;
  u64 ret_key[16];
  u64 ret_off, ret_cap;
};

// Byte offsets of the arrays in one wave's trie region.
struct IstLayout {
  size_t keys, marked, lc, ls, label, hash, path, total;
};

__host__ __device__ inline IstLayout ist_layout(int W, int k, uint32_t node_cap, u64 hslots, int drows) {
  IstLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) & ~(size_t)255;
    return r;
  };
  L.keys = take(8 * (size_t)node_cap * (size_t)W);
  L.marked = take(8 * (size_t)node_cap);
  L.lc = take(4 * (size_t)node_cap * (size_t)k);
  L.ls = take(4 * (size_t)node_cap * (size_t)k);
  L.label = take(4 * (size_t)node_cap);
  L.hash = take(8 * (size_t)hslots);
  L.path = take(4 * (size_t)k * (size_t)drows);
  L.total = o;
  return L;
}

int ist_list_launch(int W, const IstParams& prm, int grid, size_t lds, hipStream_t s);
int ist_occupancy(int W, size_t lds);
size_t ist_lds_bytes(int W, int k, int fp, int drows);
