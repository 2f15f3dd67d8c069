// pc_alpha_table.h -- alpha = y / icbrt(x) per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {
    double log10x;
    double alpha;
};

static const pc_alpha_entry kAlphaTable[] = {
    {7.0, 8}, // 0.31 ms
    {7.5, 48}, // 0.33 ms
    {8.0, 48}, // 0.35 ms
    {8.5, 48}, // 0.40 ms
    {9.0, 48}, // 0.47 ms
    {9.5, 12}, // 0.57 ms
    {10.0, 12}, // 0.74 ms
    {10.5, 12}, // 0.97 ms
    {11.0, 12}, // 1.39 ms
    {11.5, 6}, // 1.89 ms
    {12.0, 8}, // 2.59 ms
    {12.5, 8}, // 2.46 ms
    {13.0, 6}, // 2.96 ms
    {13.5, 6}, // 3.40 ms
    {14.0, 3}, // 3.66 ms
    {14.5, 2}, // 4.08 ms
    {15.0, 4}, // 5.50 ms
    {15.5, 4}, // 7.11 ms
    {16.0, 4}, // 8.92 ms
    {16.5, 12}, // 12.56 ms
    {17.0, 16}, // 24.91 ms
    {17.5, 24}, // 48.69 ms
    {18.0, 24}, // 103.71 ms
    {18.5, 32}, // 211.89 ms
    {19.0, 32}, // 457.42 ms
};
