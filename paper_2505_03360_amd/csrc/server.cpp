// placeholder; serving runtime follows
