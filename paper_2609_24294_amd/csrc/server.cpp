// server.cpp -- placeholder until the serving runtime lands
