// pc_alpha_table.h -- alpha = y / icbrt(x) and the sieve shape per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {
    double log10x;
    double alpha;       // least time for one query
    unsigned seg_kib;   // LDS segment, KiB
    unsigned wg;        // workgroup threads
    double batch_alpha; // least time for a batch of queries of this size
};

static const pc_alpha_entry kAlphaTable[] = {
    {7.0, 8, 32, 512, 2}, // 0.32 ms
    {7.5, 48, 32, 512, 1.5}, // 0.35 ms
    {8.0, 32, 64, 1024, 4}, // 0.37 ms
    {8.5, 48, 32, 512, 3}, // 0.41 ms
    {9.0, 16, 64, 1024, 4}, // 0.46 ms
    {9.5, 24, 64, 1024, 8}, // 0.51 ms
    {10.0, 48, 64, 1024, 12}, // 0.55 ms
    {10.5, 48, 64, 1024, 8}, // 0.58 ms
    {11.0, 48, 32, 512, 8}, // 1.07 ms
    {11.5, 24, 32, 512, 8}, // 1.11 ms
    {12.0, 8, 32, 512, 6}, // 1.12 ms
    {12.5, 6, 32, 512, 8}, // 1.19 ms
    {13.0, 2, 32, 512, 8}, // 1.25 ms
    {13.5, 8, 32, 512, 8}, // 1.31 ms
    {14.0, 12, 32, 512, 12}, // 1.52 ms
    {14.5, 12, 32, 512, 12}, // 2.01 ms
    {15.0, 12, 32, 512, 16}, // 2.82 ms
    {15.5, 12, 32, 512, 16}, // 4.25 ms
    {16.0, 16, 32, 512, 24}, // 6.92 ms
    {16.5, 16, 32, 512, 16}, // 11.38 ms
    {17.0, 24, 32, 512, 24}, // 23.22 ms
    {17.5, 24, 32, 512, 24}, // 44.70 ms
    {18.0, 24, 32, 512, 24}, // 98.33 ms
    {18.5, 32, 32, 512, 32}, // 205.09 ms
    {19.0, 32, 32, 512, 32}, // 431.97 ms
};
