// Plain-old-data tables shared by the host plan and the gfx950 kernels.
#pragma once
#include <stdint.h>

#define FPSSFT_MAX_STAGES 24

// Method variants (the same bits as FPSSFT_FLAG_* of the C ABI).
#define FPS_AXIS_SCHEDULE 0x1u
#define FPS_AMP_AVERAGE 0x2u
#define FPS_LITERAL_PEEL 0x4u
#define FPS_DETERMINISTIC 0x8u

// Output info words (fpssft_out.info): set size, iterations, outcome,
// detections, merged frequencies left out of the set.
#define FPS_INFO_LEN 8

// Everything a kernel needs to know about one cube. Built on the host,
// uploaded once per plan, read through scalar loads on the device.
struct CubeDesc {
  int32_t D;                 // dimensions
  int32_t L;                 // line length LCM(N_k) (Lemma 1)
  int32_t T;                 // iteration budget T_max
  int32_t max_k;             // record capacity
  int32_t dims[4];           // N_k
  int32_t c[4];              // c_k = L / N_k
  int32_t dmask[4];          // N_k - 1 when N_k is a power of two, else -1
  int64_t stride[4];         // element strides, last dimension contiguous
  int64_t N;                 // total elements
  int32_t Lmask;             // L - 1 when L is a power of two, else -1
  int32_t nstages;           // FFT stages
  int32_t radix[FPSSFT_MAX_STAGES];
  float inv_L;
  float zero_thresh;         // theta0
  float mag_rel_tol;         // rho
  float grid_tol;            // gamma (< 0: off)
  int32_t sched_off;         // int32 offset of [T][2][D] in the schedule table
  int32_t tw_off;            // float2 offset of W_L in the twiddle table
  int32_t rec_lds;           // records kept in LDS (capacity), 0: global
  int32_t serial;            // long lines, transformed one at a time through a
                             // one-line scratch, twiddles read from global memory:
                             // 1 with the spectra in LDS, 2 (longer) with the
                             // spectra and the scratch in a device workspace
  uint32_t flags;            // FPSSFT_FLAG_* of the description
  int32_t pad1;
  int64_t spec_off;          // element offset in the packed spectra buffer
  int64_t rec_off;           // byte offset of the record store in the plan's
                             // device workspace (rec_lds == 0), else -1
  int64_t lws_off;           // serial == 2: byte offset of the line workspace
                             // ((D+2) L complex values) in the same workspace,
                             // else -1
};

// Device pointers of one cube's outputs (same layout as fpssft_out).
struct OutPtrs {
  int32_t* freqs;
  void* amps;
  int32_t* rec_iter;
  int32_t* rec_bin;
  int32_t* rec_sin;
  int32_t* info;
};

// Bytes of one slot of a cube's record store (a set entry): amplitude, D
// frequency indices, canonical set index, bin-list link.
#define FPS_REC_SLOT_BYTES(D) (8 + 4 * (D) + 2 * 4)

// Largest record capacity (max_k) of a description.
#define FPS_MAX_K (1 << 26)

// Slots of the frequency hash of a record store of `cap` entries (open
// addressing with linear probing, load factor at most 1/2): the smallest
// power of two of at least 2 cap and 64; none without records.
constexpr int32_t fps_rec_hash_slots(int32_t cap) {
  int32_t h = 64;
  while (h < 2 * cap) h <<= 1;
  return cap > 0 ? h : 0;
}

// Bytes of a record store of `cap` entries: the slots, then the hash.
constexpr int64_t fps_rec_bytes(int D, int32_t cap) {
  return (int64_t)cap * FPS_REC_SLOT_BYTES(D) + 4 * (int64_t)fps_rec_hash_slots(cap);
}

// One work item of the line gather + FFT kernel: `count` iterations of one
// cube starting at t0, written at element offset `out_off`.
struct LineItem {
  int32_t cube;
  int32_t t0;
  int32_t count;
  int32_t pad;
  int64_t out_off;
};
